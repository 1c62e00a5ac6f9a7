"""On-device diagnostics built on the library's moment readout.

energy_spectrum: the kinetic-energy spectrum E(k) of the velocity field,
computed in FP64 on the GPU with a library FFT (torch.fft over rocFFT):

    u^(m) = (1/N) sum_x u(x) exp(-2 pi i m.x / n)      (m integer mode numbers)
    E(k)  = 1/2 sum over |m| in [k - 1/2, k + 1/2) of |u^(m)|^2

so that sum_k E(k) = <|u|^2> / 2 (Parseval), the kinetic energy per node of a
unit-density fluid.  Velocities are in lattice units.
"""
from __future__ import annotations

import math


def spectrum_of(u, nbins=None):
    """E(k), k = 0..nbins-1, of a velocity tensor u[D, (n,) n, n] (any torch device, FP64)."""
    import torch
    D = u.shape[0]
    shape = tuple(u.shape[1:])
    if len(shape) != D or len(set(shape)) != 1:
        raise ValueError("energy spectrum needs a cubic (square) grid")
    n = shape[0]
    N = float(n ** D)
    uh = torch.fft.fftn(u, dim=tuple(range(1, D + 1))) / N
    e = 0.5 * (uh.real ** 2 + uh.imag ** 2).sum(0)                  # per mode
    m = torch.fft.fftfreq(n, d=1.0 / n, dtype=torch.float64, device=u.device)   # integer mode numbers
    grids = torch.meshgrid(*([m] * D), indexing="ij")
    kmag = torch.sqrt(sum(g * g for g in grids))
    shell = torch.floor(kmag + 0.5).to(torch.int64)
    nb = nbins or int(math.floor(math.sqrt(D) * (n // 2) + 0.5)) + 1
    out = torch.zeros(nb, dtype=torch.float64, device=u.device)
    keep = shell < nb
    out.index_add_(0, shell[keep], e[keep])
    return out


def energy_spectrum(ctx, nbins=None):
    """E(k) of the context's current state (FP64, on the context's device);
    returns a numpy array."""
    import torch
    nodes = 1
    for s in ctx.shape:
        nodes *= s
    u = torch.empty(ctx.D * nodes, dtype=torch.float64, device="cuda")
    ctx.get_moments_device(u=u)
    ctx.sync()
    return spectrum_of(u.view((ctx.D,) + tuple(ctx.shape)), nbins).cpu().numpy()
