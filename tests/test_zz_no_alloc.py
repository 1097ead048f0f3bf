"""The no-allocation variant of vi_solve against vi_solve itself, through
the C-ABI: two calls in a row on one device (the second on a smaller MDP,
so the shared scratch memory holds the first call's contents), each
compared bit for bit with vi_solve's output on the same input, and the
rejection of an MDP whose workspace exceeds the scratch memory."""
import numpy as np
import pytest
import torch

from paper_2110_02901_amd import binding as mb
from paper_2110_02901_amd import inputs

pytestmark = pytest.mark.gpu


def dev():
    return torch.device("cuda:0")


def up(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def both(h, n, b, seed, **kw):
    """(V, V64, policy, stats) of vi_solve and of vi_solve_noalloc."""
    out = []
    for noalloc in (False, True):
        V = torch.zeros(n, dtype=torch.float32, device=dev())
        V64 = torch.zeros(n, dtype=torch.float64, device=dev())
        pol = torch.full((n,), -1, dtype=torch.int32, device=dev())
        if noalloc:
            st = mb.vi_solve_noalloc(h, V, b, seed, policy_out=pol, V64_out=V64, **kw)
        else:
            ws = mb.workspace(h, b)
            st = mb.vi_solve(h, V, b, seed, ws, policy_out=pol, V64_out=V64, **kw)
            del ws
        torch.cuda.synchronize()
        out.append((V.cpu().numpy(), V64.cpu().numpy(), pol.cpu().numpy(), st))
    return out


def check_equal(a, b):
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], b[2])
    assert a[3] == b[3] or (np.isnan(a[3]["final_err_ref"]) and np.isnan(b[3]["final_err_ref"])
                            and {k: v for k, v in a[3].items() if k != "final_err_ref"}
                            == {k: v for k, v in b[3].items() if k != "final_err_ref"})


def test_noalloc_matches_vi_solve_twice():
    # first call: dense 1024 x 16, gamma 0.99, b = 256, to max|dV| <= 1e-9
    P, c = inputs.dense_mdp(1024, 16, 0.1, 2, dtype=np.float32)
    h1 = mb.mdp_create_dense(up(P), up(c), 0.99)
    r1 = both(h1, 1024, 256, 101, tol_dv=1e-9, max_sweeps=5000)
    assert r1[0][3]["converged"] and r1[0][3]["sweeps"] > 100
    check_equal(r1[0], r1[1])
    # second call: a smaller sparse MDP (n = 500, ragged rows, CSR engine)
    rp, col, val, cc = inputs.csr_ragged_mdp(500, 3, 1, 12, 1.0, 80)
    h2 = mb.mdp_create_csr(up(rp), up(col), up(val), up(cc), 0.95)
    r2 = both(h2, 500, 37, 7, tol_dv=1e-10, max_sweeps=5000)
    assert r2[0][3]["converged"]
    check_equal(r2[0], r2[1])
    # and the first MDP once more, after the smaller one used the scratch memory
    r3 = both(h1, 1024, 1024, 5, tol_dv=-1.0, max_sweeps=40)
    assert r3[0][3]["sweeps"] == 40
    check_equal(r3[0], r3[1])


def test_noalloc_rejects_mdps_beyond_its_scratch_memory():
    # n = 400 000, m = 8, k = 4: the workspace (~38 MB) exceeds 32 MiB
    rp, col, val, c = inputs.csr_mdp(400_000, 8, 4, 1.0, 5)
    h = mb.mdp_create_csr(up(rp), up(col), up(val), up(c), 0.9)
    assert mb.mdp_workspace_bytes(h, 1000) > 32 << 20
    V = torch.zeros(400_000, dtype=torch.float32, device=dev())
    with pytest.raises(mb.MbdpError) as e:
        mb.vi_solve_noalloc(h, V, 1000, 1, tol_dv=1e-6, max_sweeps=10)
    assert e.value.status == mb.MBDP_ERR_INVALID_ARG
    assert "scratch" in str(e.value)
