"""Helpers shared by the GPU tests: build the oracle and the GPU context for
one seeded case and run both on the same conserved state."""
import numpy as np
import torch

import synth
from oracle import Oracle
from paper_2202_02319_amd import htr


def both(case, flags=None):
    o = Oracle(case, flags=flags)
    g = htr.Context.from_case(case, flags=flags)
    return o, g


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def gpu_rhs(g, U, T, t, laser, want_hrr=False):
    Ud = dev(U)
    Td = dev(T)
    out = torch.empty_like(Ud)
    hrr = torch.empty(g.N, dtype=torch.float64, device="cuda") if want_hrr else None
    htr.htr_rhs(g, Ud, Td, t, laser, out, hrr)
    htr.htr_check(g)
    return (host(out), host(Td)) + ((host(hrr),) if want_hrr else ())


def gpu_cells(g, U, T, t, laser):
    out = torch.empty((5 + 2 * g.ns + 3, g.N), dtype=torch.float64, device="cuda")
    Td = dev(T)
    htr.htr_cells(g, dev(U), Td, t, laser, out)
    htr.htr_check(g)
    return host(out)


def sub_window(case, lo, size, halo):
    """A periodic window of a larger case: cells lo-halo .. lo+size+halo-1 per
    axis (active axes only), same metrics, coordinates and laser period; the
    oracle is exact on the window interior (>= halo cells from its edge)."""
    n = case.grid.n
    idx = []
    for a in range(3):
        if n[a] == 1:
            idx.append(np.array([0]))
        else:
            idx.append(np.arange(lo[a] - halo, lo[a] + size[a] + halo) % n[a])
    g = synth.Grid(n=tuple(len(i) for i in idx), xnode=[case.grid.xnode[a][idx[a]] for a in range(3)],
                   xin=[case.grid.xin[a][idx[a]] for a in range(3)], xif=[case.grid.xif[a][idx[a]] for a in range(3)],
                   L=case.grid.L)
    flat = (idx[2][:, None, None] * n[1] + idx[1][None, :, None]) * n[0] + idx[0][None, None, :]
    flat = flat.ravel()
    sub = synth.Case(case.name + "[win]", case.mech, g, case.Y[:, flat], case.T[flat], case.p[flat],
                     case.vel[:, flat], laser=case.laser, flags=case.flags, cfl=case.cfl, theta_c=case.theta_c,
                     psi_c=case.psi_c, teno_CT=case.teno_CT)
    inner = [np.arange(halo, halo + size[a]) if n[a] > 1 else np.array([0]) for a in range(3)]
    inner_flat = ((inner[2][:, None, None] * g.n[1] + inner[1][None, :, None]) * g.n[0]
                  + inner[0][None, None, :]).ravel()
    return sub, flat, inner_flat
