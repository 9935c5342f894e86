"""Shared test helpers: run the same seeded inputs through the HIP path and
the oracle (the two never import each other)."""

import numpy as np
import torch

from oracle import step as ostep
from oracle.diagnostics import rel_l2


def setup_of(wl):
    return ostep.Setup(wl.pde, wl.dim, wl.order, wl.n_cells, wl.h, wl.pde_param,
                       wl.picard_iters)


def oracle_run(wl, Q0, par, steps, dt=None, cfl=None):
    s = setup_of(wl)
    Q = torch.tensor(Q0)
    p = None if par is None else torch.tensor(par)
    Q, dts = ostep.run(Q, p, s, steps, cfl=cfl, dt=dt)
    return Q, dts


def gpu_run(wl, Q0, par, steps, dt=None, cfl=None, record_dt=False):
    from paper_1801_08682_amd.stepper import Stepper
    st = Stepper(wl)
    Q = torch.tensor(Q0, device="cuda")
    p = None if par is None else torch.tensor(par, device="cuda")
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    rec = st.run(Q, p, steps, cfl=cfl, dt=dt, flag=flag, record_dt=record_dt)
    torch.cuda.synchronize()
    out = Q.cpu()
    dts = [float(x.item()) for x in rec]
    st.close()
    return out, int(flag.item()), dts


def max_rel(Q, ref, wl):
    return float(rel_l2(Q, ref, setup_of(wl)).max())


def per_field(Q, ref, wl):
    return [float(x) for x in rel_l2(Q, ref, setup_of(wl))]
