"""Race check for the sparse engines: a state's backup is computed the same
way whichever workgroup computes it (a wavefront per state, its row in a
fixed lane order, reductions in a fixed order), so the result of a solve
must not depend on the grid.  Solves with 256 workgroups of 1024 threads and
with 512 of 512 -- a different assignment of states, chunks and batches to
workgroups, a different barrier, different timing -- must agree bit for bit
(VI and MB-MPI, Algorithm 1, at small, ragged and full batches).  The dense
engine is left out: its grouping of a row's columns follows the grid, so
its rounding does too."""
import numpy as np
import pytest
import torch

from paper_2110_02901_amd import binding as mb
from paper_2110_02901_amd import inputs

from gpu_util import csr_case, dev

pytestmark = pytest.mark.gpu

GRIDS = ((1, 1024), (2, 512))  # (workgroups per CU, threads per workgroup)


def solve(h, n, b, grid, mpi):
    mb.mdp_set_tuning(h, blocks_per_cu=grid[0], threads_per_block=grid[1],
                      band_window=getattr(h, "_test_band_window", 0))
    ws = mb.workspace(h, b)
    V = torch.zeros(n, dtype=torch.float32, device=dev())
    if mpi:
        pol = torch.zeros(n, dtype=torch.int32, device=dev())
        st = mb.mpi_solve(h, V, pol, 3, b, 17, ws, policy_is_init=False, tol_dv=-1.0,
                          max_outer=6)
        return V.cpu().numpy(), pol.cpu().numpy(), st
    st = mb.vi_solve(h, V, b, 17, ws, tol_dv=-1.0, max_sweeps=25)
    return V.cpu().numpy(), None, st


def cases():
    n, m = 3000, 8
    rp, col, val, c = inputs.csr_mdp(n, m, 32, 1.0, 61, band=None)
    ell, _ = csr_case(rp, col, val, c, 0.99)
    ell._test_band_window = -1  # the plain ELL engine
    rp, col, val, c = inputs.csr_mdp(n, m, 32, 1.0, 62, band=64)
    band, _ = csr_case(rp, col, val, c, 0.99)
    rp, col, val, c = inputs.csr_ragged_mdp(n, m, 1, 40, 1.0, 63)
    csr, _ = csr_case(rp, col, val, c, 0.99)
    return n, {"ell": ell, "ell-band": band, "csr": csr}


@pytest.fixture(scope="module")
def handles():
    n, hs = cases()
    yield n, hs
    for h in hs.values():
        h.close()


@pytest.mark.parametrize("kind", ["ell", "ell-band", "csr"])
@pytest.mark.parametrize("b", [7, 300, 3000])
@pytest.mark.parametrize("mpi", [False, True])
def test_solve_does_not_depend_on_the_grid(handles, kind, b, mpi):
    n, hs = handles
    h = hs[kind]
    runs = [solve(h, n, b, g, mpi) for g in GRIDS]
    mb.mdp_set_tuning(h, band_window=getattr(h, "_test_band_window", 0))
    assert mb.mdp_engine(h, b) == kind
    V0, V1 = runs[0][0], runs[1][0]
    assert runs[0][2]["sweeps"] == runs[1][2]["sweeps"] > 0
    assert np.array_equal(V0.view(np.uint32), V1.view(np.uint32)), \
        "max abs difference %.3g" % float(np.max(np.abs(V0 - V1)))
    if mpi:
        assert np.array_equal(runs[0][1], runs[1][1])
