"""Shared helpers of the GPU tests: layout conversion between the library's
f[a][y][x] device tensors and the oracle's f[y, x, a] arrays, and parameter
mirroring.  No arithmetic of the method lives here."""
import numpy as np

from oracle import stepper as ostep


def to_oracle(f):
    """(9, ny, nx) tensor -> (ny, nx, 9) float64 C-contiguous numpy array."""
    a = f.detach().to("cpu").double().numpy()
    return np.ascontiguousarray(np.moveaxis(a, 0, 2))


def to_device(f, torch_dtype, device="cuda"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.moveaxis(f, 2, 0))).to(device=device, dtype=torch_dtype)


def oracle_params(p):
    """Oracle parameters equal to the library's lbm_params p."""
    s = (p.s_rho, p.s_e, p.s_zeta, p.s_j, p.s_q, p.s_j, p.s_q, p.s_nu, p.s_nu)
    return ostep.make_params(p.nx, p.ny, p.T, walls=bool(p.walls_y), a=p.a, b=p.b, R=p.R, G=p.G,
                             eps=p.eps, s=s)


def rel_inf(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
