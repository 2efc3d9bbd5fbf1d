"""Helpers for the GPU parity tests: run the HIP path and the oracle on the
same seeded workload and compare."""
import numpy as np
import torch

import oracle

DEV = torch.device("cuda:0") if torch.cuda.is_available() else None
TOL_MOMENT = 1e-10  # |mu| <= 1, so this is relative as well


def gpu_moments(w, sites=None, N=None, tile=None, precision=0, fixed=None, algorithm=0):
    import paper_1007_1609_amd as P
    op = P.Operator.from_workload(w, DEV, fixed=fixed)
    s = w.start_sites if sites is None else np.asarray(sites, dtype=np.int32)
    st = torch.as_tensor(s, dtype=torch.int32, device=DEV)
    mu_ee, mu_he = P.chebyshev_moments(op, st, w.N if N is None else N,
                                       (w.tile if tile is None else tile), precision,
                                       algorithm=algorithm)
    torch.cuda.synchronize()
    return op, mu_ee.cpu().numpy(), mu_he.cpu().numpy()


def oracle_moments(w, a, b, sites=None, N=None):
    return oracle.workload_moments(w, a, b, sites=sites, N=N)


def maxdiff(x, y):
    return float(np.max(np.abs(np.asarray(x) - np.asarray(y)))) if np.size(x) else 0.0
