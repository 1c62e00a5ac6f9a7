/*
 * cmlb: central-moment multiple-relaxation-time lattice Boltzmann on MI355X.
 *
 * C ABI of the library that advances the fused pull-stream-and-collide update
 * of X. Shan, "A central-moment multiple-relaxation-time collision model"
 * (arXiv:1808.04406) on a periodic grid, on one AMD Instinct GPU (gfx950).
 *
 * The update (Sec. II.C, final equation) is f_i(x + xi_i, t + 1) = f^_i + Omega_i:
 * every node gathers its populations, forms rho, u (and theta on the thermal
 * lattice), relaxes each order n of central moments at its own rate omega_n
 * = 1/tau_n (eq:omega), maps the result back to the absolute frame on the
 * fixed velocities (eq:mrt, eq:fi) and stores the post-collision populations.
 *
 * Conventions shared by every call:
 *  - Lattices (the quadrature of eq:quad, xi_i = r e_i):
 *      CMLB_D2Q9   e in {-1,0,1}^2, r = sqrt(3), complete tensor-product basis;
 *      CMLB_D3Q27  e in {-1,0,1}^3, r = sqrt(3), complete tensor-product basis;
 *      CMLB_D2Q37  e in Z^2 with |e|^2 <= 10, ninth-degree rule (r ~ 1.19698),
 *                  order-4 Hermite truncation N = M = 4 (Sec. II.B);
 *      the other 2D Hermite rules of Fig. 2 (see the lattice enum).
 *    Population order: D2Q9/D3Q27 i = (ex+1) + 3(ey+1) + 9(ez+1); the 2D
 *    Hermite rules lexicographic in (ey, ex), both from -3 to 3.
 *  - Host arrays of fields and populations are FP64, structure of arrays,
 *    x fastest: fields [component][z][y][x], populations [i][z][y][x].
 *    Velocities are in lattice units (cells per step); theta is the paper's
 *    dimensionless temperature (1 is the lattice reference).
 *  - The state is the post-collision population field; one step pulls
 *    f_i(x - e_i) and collides (the paper's push update re-indexed).
 *  - Every function returns CMLB_OK (0) or a negative error code; a failing
 *    call leaves the context unchanged and cmlb_last_error() describes it.
 *    No C++ exception crosses this interface.
 *  - Ownership: the library never keeps a host pointer after a call returns.
 *    It owns the device buffers it allocates; buffers passed to
 *    cmlb_create_external stay owned by the caller and must outlive the
 *    context.
 */
#ifndef CMLB_H
#define CMLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CMLB_OK 0
#define CMLB_EINVAL (-1)    /* bad argument */
#define CMLB_ENOMEM (-2)    /* device or host allocation failed */
#define CMLB_EDEVICE (-3)   /* HIP runtime or kernel launch error */
#define CMLB_ESTATE (-4)    /* call not valid in the current state */
#define CMLB_EUNSTABLE (-5) /* non-finite populations found (divergence) */

/* Lattices.  The 2D Hermite rules (eq:quad, Sec. III.A and Fig. 2) are the
 * minimal on-lattice rules whose velocity components are at most 3: four of
 * degree 9 on 37 velocities, carrying the order-4 truncation N = M = 4
 * (CMLB_D2Q37 is the one on the shells with |e|^2 <= 10, also called E9 A),
 * and four of degree 7 on 17 velocities, carrying N = M = 3 (a degree-7 rule
 * resolves the Hermite coefficients of eq:an exactly only up to order
 * 7 - N).  Their shells, as |e| component pairs beside the rest velocity:
 *   CMLB_D2Q37 (E9 A)  (0,1) (1,1) (0,2) (1,2) (2,2) (0,3) (1,3)
 *   CMLB_E9B           (0,1) (1,1) (0,2) (1,2) (2,2) (0,3) (2,3)
 *   CMLB_E9C           (0,1) (1,1) (0,2) (1,2) (3,3) (0,3) (1,3)
 *   CMLB_E9D           (0,1) (1,1) (0,2) (1,2) (3,3) (0,3) (2,3)
 *   CMLB_E7A           (0,1) (1,1) (2,2) (0,3)
 *   CMLB_E7B           (0,1) (1,1) (3,3) (0,3)
 *   CMLB_E7C           (0,2) (1,1) (3,3) (0,3)
 *   CMLB_E7D           (1,1) (2,2) (3,3) (0,3)
 * The letters order the rules by their shells; the paper does not print its
 * tables.  The rules other than D2Q37 take FP64 or FP32 storage, the
 * central-moment or the regularised BGK model, and one step per launch. */
enum { CMLB_D2Q9 = 0, CMLB_D3Q27 = 1, CMLB_D2Q37 = 2, CMLB_E9B = 3, CMLB_E9C = 4, CMLB_E9D = 5,
       CMLB_E7A = 6, CMLB_E7B = 7, CMLB_E7C = 8, CMLB_E7D = 9 };

/* Storage of the population field.  Every type stores the deviation
 * g_i = s_i (f_i - w_i rho0); arithmetic is FP64 for CMLB_F64 and FP32 for
 * the others.  The automatic s_i is a power of two: 1 for F64/F32/BF16, and
 * for F16 chosen from w_i so that |f_i - w_i rho0| up to 8 w_i stays
 * representable (cmlb_params.scale overrides it). */
enum { CMLB_F64 = 0, CMLB_F32 = 1, CMLB_BF16 = 2, CMLB_F16 = 3 };

/* Collision model.  CMLB_MODEL_CM is the paper's central-moment MRT
 * (eq:omega, eq:mrt).  The two others are the comparison operators of
 * eq:regnmrt: raw-moment MRT relaxes absolute-frame Hermite coefficients at
 * per-order rates, regularised BGK (eq:lbgk-reg) relaxes every order at
 * omega_2.  Raw MRT is available on CMLB_D2Q37, regularised BGK on every 2D
 * Hermite rule. */
enum { CMLB_MODEL_CM = 0, CMLB_MODEL_RAW_MRT = 1, CMLB_MODEL_REG_BGK = 2 };

typedef struct cmlb_params {
    int32_t lattice;   /* CMLB_D2Q9, CMLB_D3Q27, CMLB_D2Q37, CMLB_E9B..CMLB_E7D */
    int32_t storage;   /* CMLB_F64, CMLB_F32, CMLB_BF16, CMLB_F16 */
    int32_t model;     /* CMLB_MODEL_* */
    int32_t thermal;   /* 1: theta follows from f (2D Hermite rules only); 0: theta frozen at theta0 */
    int64_t nx, ny, nz;/* periodic grid, each 1..2^20; nz must be 1 for 2D
                          lattices; the 2D Hermite rules need nx, ny >= 3
                          (their velocities reach 3 cells); nx*ny*nz < 2^32
                          and Q*nx*ny*nz < 2^35 */
    double rho0;       /* reference density of the deviation storage (>0, finite) */
    double theta0;     /* frozen temperature of isothermal runs (>0, finite) */
    double tau[8];     /* tau[n]: relaxation time of central-moment order n
                          (n >= 2; entries 0 and 1 ignored; 0 means 1.0,
                          otherwise > 0 and finite) */
    double scale[37];  /* storage scale s_i per population (entries beyond Q
                          ignored); 0 means automatic, otherwise > 0 and
                          finite */
    int32_t device;    /* HIP device ordinal */
    int32_t reserved;  /* must be 0 */
    void *hip_stream;  /* hipStream_t for all work, or NULL for a library stream */
} cmlb_params;

/* Global FP64 diagnostics of the current state (Sec. III.B's kinetic-energy
 * history and the conservation checks).  momentum and energy are in lattice
 * units: sum f e and sum f |e|^2 / 2; kinetic_energy = sum rho |u|^2 / 2;
 * enstrophy = sum |curl u|^2 / 2 with second-order central differences
 * (2D: the single vorticity component). */
typedef struct cmlb_globals {
    double mass;
    double momentum[3];
    double energy;
    double kinetic_energy;
    double enstrophy;
    int64_t n_nonfinite;
    double rho_min, rho_max; /* smallest and largest node density (finite nodes) */
    double u_max;            /* largest |u| (lattice units, finite nodes) */
} cmlb_globals;

typedef struct cmlb_ctx cmlb_ctx;

/* Lattice table (eq:quad): D, Q, e[Q*3] (integers), w[Q], r.  Any output
 * pointer may be NULL.  Host-only; needs no device. */
int cmlb_lattice_info(int lattice, int *D, int *Q, int *e, double *w, double *r);

/* Achievable HBM bandwidth for the step's access pattern, the measured
 * ceiling beside the 8 TB/s peak (a measurement aid; the paper has no
 * counterpart).  Copies `planes`
 * (1 or 27) FP32 planes filling `bytes` from one device buffer to another,
 * one element of every plane per thread as the step kernels do, `reps`
 * times after one warm-up copy, and writes (read + written bytes) / time in
 * GB/s to *gbps.  Allocates and frees its two buffers and its stream;
 * synchronises.  CMLB_EINVAL for bad arguments, CMLB_ENOMEM if the buffers
 * do not fit, CMLB_EDEVICE on a device error. */
int cmlb_copy_bandwidth(int device, uint64_t bytes, int planes, int reps, double *gbps);

/* Layout of the population state (device memory, storage type): structure
 * of arrays, population i of node (x, y, z) at
 *     i * plane + (z * ny + y) * pitch + x,
 * where pitch is nx rounded up to a multiple of 128 bytes, or nx itself when
 * that would add more than one eighth (so every x-row of a large grid starts
 * on a 128-byte line, which the pulls need to stream at full rate).  D3Q27
 * FP32 states whose rows are already a multiple of 32 bytes (nx % 8 == 0)
 * are not padded: their default two-step kernel streams such rows at full
 * rate.  plane is pitch * ny * nz, except for D3Q27 states in BF16 or FP16
 * storage, whose planes of at least 1 MiB are padded to their byte size
 * rounded up to 8 KiB plus 4 KiB, so that the 27 planes, streamed together,
 * start 4 KiB apart modulo 8 KiB (their one-step kernel runs 3 % faster so
 * at 512^3; the FP32 and FP64 two-step kernels and the 2D row sweeps were
 * no faster or slower).  Padding entries are never read; the library
 * zeroes its own buffers once at creation.
 * cmlb_state_layout gives pitch and plane, cmlb_state_bytes (Q * plane
 * elements) the buffer size.
 * Host-side arrays (fields, cmlb_get/set_populations, training batches, the
 * box filter's output) are unpadded, [component][z][y][x]. */

/* Bytes of one population buffer for parameters p (validated as by
 * cmlb_create; host only, no device needed).  Sizes the buffers of
 * cmlb_create_external. */
int cmlb_state_bytes(const cmlb_params *p, size_t *bytes);

/* Row pitch and population-plane stride, in elements, of the state for
 * parameters p (layout of the state above; validated as by cmlb_create;
 * host only).  CMLB_EINVAL for NULL outputs or invalid parameters. */
int cmlb_state_layout(const cmlb_params *p, uint64_t *pitch, uint64_t *plane);

/* Create a context: validates p, allocates two population buffers of
 * cmlb_state_bytes bytes on p->device.  The state is
 * undefined until cmlb_init_fields or cmlb_set_populations.
 * What the parameters fix, and where the paper defines it:
 *  - p->lattice: the abscissas xi_i and weights w_i of an on-lattice
 *    quadrature rule (Sec. II.A, eq:quad), on which eq:an and eq:fi are an
 *    exact transform between populations and Hermite coefficients;
 *  - p->tau[n]: the relaxation time of central-moment order n, omega_n =
 *    1 / tau_n (Sec. II.C, eq:omega; eq:mrt spells it out for n <= 4);
 *  - p->thermal: whether theta follows from the populations or stays at
 *    p->theta0 in the equilibrium (the isothermal runs of Sec. III.B);
 *  - p->model: the central-moment operator, or the raw-moment MRT and
 *    regularised BGK operators it is compared with (Sec. II.B-C, eq:regnmrt,
 *    eq:lbgk-reg).
 * The truncation orders are fixed per lattice (N = M = 4 on D2Q37 as in all
 * of Sec. III; the complete basis on D2Q9 and D3Q27).  On failure
 * *out is NULL and cmlb_create_error() describes the reason: CMLB_EINVAL
 * for parameters outside the ranges documented in cmlb_params (checked
 * before any device call), CMLB_EDEVICE or CMLB_ENOMEM from the device. */
int cmlb_create(const cmlb_params *p, cmlb_ctx **out);

/* As cmlb_create, but the population buffers f_a and f_b are device memory
 * owned by the caller (for example PyTorch tensors), each at least
 * cmlb_state_bytes bytes, 256-byte aligned and not overlapping (a step reads
 * one and writes the other); CMLB_EINVAL otherwise. */
int cmlb_create_external(const cmlb_params *p, void *f_a, void *f_b, cmlb_ctx **out);

/* Reason for the last failed create on this thread. */
const char *cmlb_create_error(void);

/* Free the library-owned device memory and the context.  NULL is a no-op. */
void cmlb_destroy(cmlb_ctx *ctx);

/* Description of the last error on ctx ("" if none). */
const char *cmlb_last_error(const cmlb_ctx *ctx);

/* Replace tau_n for orders 2 .. 2+n-1 (tau_by_order[k] is tau of order k+2;
 * host array of n values, 1 <= n <= 6, each > 0 and finite, else
 * CMLB_EINVAL).  Central moments of order n relax at omega_n = 1 / tau_n
 * (Sec. II.C, eq:omega, required there for every order n); orders 0 and 1
 * are conserved and have no rate.  Takes effect at the next cmlb_step. */
int cmlb_set_tau(cmlb_ctx *ctx, const double *tau_by_order, int n);

/* Set the state to the discrete equilibrium of the given fields (host FP64,
 * rho[node], u[D][node], theta[node] or NULL for theta0): the complete-basis
 * equilibrium on D2Q9/D3Q27, the order-4 Hermite equilibrium on D2Q37
 * (Sec. II.B, eq:maxwellian truncated). */
int cmlb_init_fields(cmlb_ctx *ctx, const double *rho, const double *u, const double *theta);

/* As cmlb_init_fields with the fields already in device memory. */
int cmlb_init_fields_device(cmlb_ctx *ctx, const double *rho, const double *u, const double *theta);

/* Enqueue n stream-and-collide steps on the context stream (asynchronous).
 * One step is the update of Sec. II.C (its final equation,
 * f_i(x + xi_i, t + 1) = f^_i + Omega_i, with f^ the projection of eq:reg
 * and Omega the central-moment relaxation of eq:omega / eq:mrt) on the
 * periodic grid, written as a pull: every node gathers f_i(x - e_i) and
 * collides.  n >= 0 (n = 0 does nothing); CMLB_ESTATE before the state is
 * initialised.  Divergence is not checked here (see cmlb_reduce).  On D3Q27 with FP32 or FP64 storage and on D2Q37 with FP32 storage
 * (learned closure off) pairs of steps run as one launch that keeps the
 * intermediate state on chip; the result is identical to single steps (see
 * cmlb_set_step_fusion). */
int cmlb_step(cmlb_ctx *ctx, int64_t n);

/* Steps per kernel launch for cmlb_step.  Two steps per launch are
 * supported on D3Q27 with FP32 or FP64 storage (learned closure off,
 * population planes below 2 GiB) and on D2Q37 with FP32 storage (every
 * collision model, state below 4 GiB); elsewhere every value launches one
 * kernel per step.
 *   0 (default)  automatic: two steps per launch where supported, unless a
 *                cost model of the grid's launch shape expects two single
 *                launches to be faster (small grids);
 *   1            one kernel per step;
 *   2            two steps per launch wherever supported;
 *   3            as 2, but D2Q37 runs the kernel that folds each first-step
 *                row into the moments of the second-step rows it feeds
 *                (one row in LDS, two waves per SIMD).  Its moment sums run
 *                in another order, so it equals two single steps to FP32
 *                rounding, not bitwise; on one MI355X it is no faster
 *                (1024^2: 21,500 against 21,700 MLUPS; 2048^2: 23,000
 *                against 24,600).
 * Modes 0, 1 and 2 give bitwise the same populations.  CMLB_EINVAL for
 * other values. */
int cmlb_set_step_fusion(cmlb_ctx *ctx, int steps_per_launch);

/* Replay the steps of cmlb_step from a HIP graph of `steps` steps (a
 * positive multiple of 4; 0, the default, launches every kernel directly).
 * The graph is captured on the context stream at the first cmlb_step of at
 * least `steps` steps and replayed n / steps times; the remaining steps are
 * launched directly.  Results are bitwise those of direct launches.  The
 * graph is recaptured after cmlb_set_tau, cmlb_set_step_fusion and
 * cmlb_closure_enable, and whenever the buffer parity differs from the
 * captured one.  On one MI355X replay is no faster than direct launches
 * (the device, not the host, sets the pace of short launches); it serves
 * callers that drive steps from graphs of their own.
 * CMLB_EINVAL for other values. */
int cmlb_set_graph_steps(cmlb_ctx *ctx, int steps);

/* Most contexts one cmlb_step_batch call can step together. */
#define CMLB_MAX_BATCH 16

/* Enqueue n steps of each of `count` contexts (1..CMLB_MAX_BATCH, distinct),
 * one launch per step for all of them: many small lattices fill the GPU
 * that one alone would leave mostly idle (Sec. III.B: the stability search
 * runs hundreds of 128^2 lattices).  The contexts must agree in lattice,
 * storage, collision model, thermal flag, grid, rho0, theta0, storage scales
 * and device, and have the learned closure off; relaxation times, buffer
 * parities and streams may differ.  Each context's populations and step
 * count end exactly as after cmlb_step(ctx, n) with one step per launch
 * (which gives the same populations as any fusion setting).  Asynchronous:
 * the launches go on ctxs[0]'s stream after the work already enqueued on
 * the other contexts' streams, and work enqueued later on any of those
 * streams runs after them.  If validation fails nothing is enqueued (the
 * message is on ctxs[0]); CMLB_EINVAL if ctxs or ctxs[0] is NULL or
 * count < 1. */
int cmlb_step_batch(cmlb_ctx *const *ctxs, int count, int64_t n);

/* Wait for all work enqueued on the context stream. */
int cmlb_sync(cmlb_ctx *ctx);

/* Read rho[node], u[D][node] (lattice units) and theta[node] of the state
 * (host FP64; any pointer may be NULL).  Synchronises.  These are the
 * leading moments of Sec. II.A (the equation after eq:fi): rho = sum f_i,
 * rho u = sum f_i xi_i, rho (u^2 + D theta) = sum f_i xi_i^2 with
 * xi_i = r e_i; u is returned divided by r (cells per step).  On
 * isothermal contexts theta is theta0.  Caller-owned arrays of nx*ny*nz
 * (rho, theta) and D*nx*ny*nz (u) doubles. */
int cmlb_get_moments(cmlb_ctx *ctx, double *rho, double *u, double *theta);

/* As cmlb_get_moments into caller-owned device arrays (FP64, same layout;
 * any pointer may be NULL), enqueued on the context stream without waiting:
 * order later work on that stream or call cmlb_sync.  Used for on-device
 * diagnostics such as the kinetic-energy spectrum. */
int cmlb_get_moments_device(cmlb_ctx *ctx, double *rho, double *u, double *theta);

/* Read / write the full populations f_i (decoded, host FP64, [i][node]).
 * Writing encodes to the storage type (round to nearest even). Synchronises. */
int cmlb_get_populations(cmlb_ctx *ctx, double *f);
int cmlb_set_populations(cmlb_ctx *ctx, const double *f);

/* FP64 global diagnostics of the state (deterministic two-pass reduction).
 * Returns CMLB_EUNSTABLE (with *out filled) if any population is not finite. */
int cmlb_reduce(cmlb_ctx *ctx, cmlb_globals *out);

/* ---- Allocation-free diagnostics ----------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  Computes
 * exactly what cmlb_reduce computes, with the same kernels, but keeps their
 * scratch (the FP64 velocity field of the enstrophy pass, the per-block
 * partial sums and the final sums) in a fixed device array of
 * CMLB_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs
 * on until the process ends; it calls no hipMalloc or hipFree.  Grids of at
 * most CMLB_NOALLOC_MAX_NODES nodes (for example 128^3, or 1536^2); larger
 * grids get CMLB_EINVAL and nothing is launched.  All calls on one device
 * share its array: calls that overlap on one GPU (from several host
 * threads) race, and the caller must serialise them.  Every entry of the
 * array is written before it is read, so no call depends on what an earlier
 * one left there.  Synchronises the context stream; returns CMLB_EUNSTABLE
 * like cmlb_reduce. */
#define CMLB_NOALLOC_SCRATCH_BYTES (64u << 20)
#define CMLB_NOALLOC_MAX_NODES 2621440
int cmlb_reduce_noalloc(cmlb_ctx *ctx, cmlb_globals *out);

/* Device pointer and byte size of the current population buffer, and the
 * stream the library launches on (hipStream_t). */
int cmlb_state(cmlb_ctx *ctx, void **f_cur, size_t *bytes, void **hip_stream);

/* Number of steps taken since the last init or set. */
int64_t cmlb_step_count(const cmlb_ctx *ctx);

/* Set the step counter (a resumed checkpoint continues its count).
 * CMLB_EINVAL for negative values. */
int cmlb_set_step_count(cmlb_ctx *ctx, int64_t steps);

/* Relaxation times in use, indexed by order: tau[n] for n = 0..7 (entries 0
 * and 1 are unused; 0 means the default 1).  Host array of 8 doubles. */
int cmlb_get_tau(const cmlb_ctx *ctx, double *tau);

/* Storage scale s_i actually in use (Q values). */
int cmlb_get_scale(const cmlb_ctx *ctx, double *scale);

/* Copy the current population buffer to / from device memory in the
 * context's own layout and storage type (cmlb_state_bytes bytes, rows
 * and planes padded as in the layout of the state).  Loading marks the state initialised and resets the
 * step count. */
int cmlb_store_state_device(cmlb_ctx *ctx, void *dst);
int cmlb_load_state_device(cmlb_ctx *ctx, const void *src);

/* Load the state from FP32 deviations f_i - w_i rho0 in device memory,
 * unpadded [i][z][y][x] (Q * nx * ny * nz floats: the layout of the box
 * filter's output and of training batches), encoded into the context's
 * storage type (times its scale s_i) and layout.  Asynchronous on the
 * context stream; marks the state initialised and resets the step count.
 * The caller keeps ownership of src, which must stay valid until the
 * stream has run the copy. */
int cmlb_load_deviations_device(cmlb_ctx *ctx, const float *src);

/* Box filter for coarse-graining (D3Q27 contexts): the populations of
 * factor^3 blocks of nodes are averaged (a linear filter, so mass and
 * momentum are kept) and written to dst as FP32 deviations f_i - w_i rho0
 * on the (nx/factor, ny/factor, nz/factor) grid, layout [i][z][y][x].
 * nx, ny, nz must be multiples of factor. */
int cmlb_box_filter(cmlb_ctx *ctx, int factor, void *dst);

/* ---- Learned closure (D3Q27 contexts with FP32 storage) ----------------
 * Not part of the paper: a per-node network sets the rates omega_3..omega_6
 * of eq:omega.  Inputs: x_p = (kappa_p - kappa_eq,p) / (rho sigma_p) for the
 * 27 central moments p = px + 3 py + 9 pz (lattice units); network
 * 27 -> GELU 32 -> GELU 32 -> 4, omega_{3+j} = 0.5 + 1.45 sigmoid(z_j).
 * Parameters: 2084 FP32 values W1[32][27], b1[32], W2[32][32], b2[32],
 * W3[4][32], b3[4] (row-major [out][in]); the step evaluates the network
 * with BF16 weights and activations and FP32 accumulation (matrix cores). */
#define CMLB_CLOSURE_NPARAM 2084

/* Load FP32 parameters (kept as the FP32 master copy) and the 27 input
 * scales sigma_p (> 0); resets the optimiser state.  Host arrays. */
int cmlb_closure_load(cmlb_ctx *ctx, const float *params, const float *sigma);

/* Use (1) or stop using (0) the network rates in cmlb_step. */
int cmlb_closure_enable(cmlb_ctx *ctx, int on);

/* With on = 1, orders 4 and 6 relax at omega_2 instead of the network's
 * rates (its outputs 1 and 3 are then unused and get no gradient).  A
 * central monomial of order 4 or 6 carries second-order Hermite content, and
 * rates differing from omega_2 make the linearised update grow as
 * tau_2 -> 1/2; the network's range [0.5, 1.95] cannot reach omega_2 there.
 * Default 0.  Needs a loaded closure; kept across cmlb_closure_load. */
int cmlb_closure_tie_even(cmlb_ctx *ctx, int on);

/* Current FP32 master parameters (host array of 2084). */
int cmlb_closure_get(cmlb_ctx *ctx, float *params);

/* A training batch: n_pairs consecutive (state, target) pairs in device
 * memory, each Q * nx*ny*nz FP32 deviations, unpadded [i][z][y][x] (the
 * box filter's output layout).  The
 * state is pulled (streamed) and collided with the network's rates.  Under
 * the default objective the target is the state one coarse step later and
 * the objective is the mean over all nodes of sum_i (f*_i - fbar_i)^2 / w_i;
 * under CMLB_CLOSURE_OBJ_MOMENTUM the target is the state two coarse steps
 * later and only its momentum is compared (cmlb_closure_set_objective).
 * nx must be a multiple of 64. */
typedef struct cmlb_batch {
    const void *state;
    const void *target;
    int64_t n_pairs;
} cmlb_batch;

/* Objective and its gradient (host outputs; grad may be NULL). */
int cmlb_closure_objective(cmlb_ctx *ctx, const cmlb_batch *batch, float *objective, float *grad);

/* One Adam step with learning rate lr on the batch objective (moments kept
 * on the device and reset by cmlb_closure_load); *objective receives its
 * value before the update. */
int cmlb_closure_train_step(cmlb_ctx *ctx, const cmlb_batch *batch, float lr, float *objective);

/* Adam's constants for cmlb_closure_train_step (training infrastructure, not
 * in the paper): P -= lr mhat / (sqrt(vhat) + eps), m = beta1 m + (1 - beta1) g,
 * v = beta2 v + (1 - beta2) g^2, mhat and vhat divided by 1 - beta^t at step
 * t.  Defaults 0.9, 0.999, 1e-8.  The objectives scale with the flow's
 * amplitude and the grid (the momentum objective is about 1e-12 on 128^3
 * from 512^3 at Mach 0.09), and eps must lie well below sqrt(vhat), the
 * gradient's size, or it shrinks every step.  beta1, beta2 in [0, 1); eps a
 * positive normal FP32 number; else CMLB_EINVAL and nothing changes.  Kept
 * across cmlb_closure_load.  Applies from the next step. */
int cmlb_closure_set_adam(cmlb_ctx *ctx, double beta1, double beta2, double eps);

/* Outputs whose weights cmlb_closure_train_step leaves unchanged (training
 * infrastructure, not in the paper): bit j (0..3) of mask freezes the rate
 * of order 3 + j, i.e. row j of W3 and b3[j], and their Adam moments.  With
 * that row of W3 zero the order's rate stays the constant its b3 entry
 * gives.  An order whose rate moves the objective little can still be
 * driven by Adam (whose steps do not shrink with the gradient) into rates
 * that are linearly unstable, e.g. omega_5 near 1.95 with omega_3 near 0.5.
 * mask in [0, 15], else CMLB_EINVAL.  Default 0; kept across
 * cmlb_closure_load. */
int cmlb_closure_freeze(cmlb_ctx *ctx, int mask);

/* Objective of cmlb_closure_objective and cmlb_closure_train_step (not in
 * the paper; default CMLB_CLOSURE_OBJ_POPULATIONS):
 *   CMLB_CLOSURE_OBJ_POPULATIONS  the population mismatch described with
 *       cmlb_batch, the target being the state one coarse step later;
 *   CMLB_CLOSURE_OBJ_MOMENTUM  the momentum two coarse steps ahead, the
 *       target being the state two coarse steps later: the state is
 *       streamed and collided with the network's rates (f1), streamed once
 *       more, and the objective is the mean over nodes of
 *       |sum_i e_i f1_i(x - e_i) - sum_i e_i target_i(x)|^2 (the second
 *       collision conserves momentum).  The library keeps two device
 *       buffers of 27 and 3 FP32 values per node and pair for it.
 * The one-step population mismatch is dominated by the non-equilibrium
 * part of the populations, which scales with the lattice spacing; the
 * momentum carries none.  CMLB_EINVAL for other values. */
#define CMLB_CLOSURE_OBJ_POPULATIONS 0
#define CMLB_CLOSURE_OBJ_MOMENTUM 1
int cmlb_closure_set_objective(cmlb_ctx *ctx, int kind);

#ifdef __cplusplus
}
#endif

#endif /* CMLB_H */
