"""J* of a sparse MDP as a differentiable torch function.

The forward pass is MB-MPI on the library (K sweeps of B_{mu,b} per
improvement, Algorithm 1) until the policy is stable and the Bellman
residual is below `tol`; it returns J* in FP64.  The backward pass uses the
optimal policy mu: near the data J* = (I - gamma P_mu)^-1 c_mu (eq. (4)),
so for an upstream gradient g = dL/dJ* the adjoint lambda = (I - gamma
P_mu)^-T g gives dL/dc(s, a) = lambda(s) [a == mu(s)] and dL/dP(s, a, s') =
gamma lambda(s) J*(s') [a == mu(s)].  lambda is computed by the same
mini-batch sweep on the transposed policy rows (library calls
mdp_policy_transpose, vi_solve with m = 1, mdp_value_gradients).  The
gradients are exact where the optimal policy is unique; at ties among
optimal actions J* is not differentiable.
"""
import torch

from . import binding as mb


class OptimalValue(torch.autograd.Function):
    """J* = OptimalValue.apply(c, val, row_ptr, col, gamma, b, seed, tol, K).

    c: FP32 [n, m] costs; val: FP32 [n*m*k] transition values with a
    constant row length k (row_ptr int64 [n*m+1], col int32 [n*m*k]).
    Gradients flow to c and val.
    """

    @staticmethod
    def forward(ctx, c, val, row_ptr, col, gamma, b=None, seed=0, tol=1e-10, K=5):
        n, m = c.shape
        k = col.numel() // (n * m)
        b = n if b is None else int(b)
        h = mb.mdp_create_csr(row_ptr, col, val.detach(), c.detach(), gamma)
        ws = mb.workspace(h, b)
        V = torch.zeros(n, dtype=torch.float32, device=c.device)
        V64 = torch.zeros(n, dtype=torch.float64, device=c.device)
        pol = torch.zeros(n, dtype=torch.int32, device=c.device)
        st = mb.mpi_solve(h, V, pol, K, b, seed, ws, policy_is_init=False, tol_dv=tol,
                          max_outer=100000, V64_out=V64)
        if not st["converged"]:
            raise RuntimeError("MB-MPI did not converge: %s" % st)
        ctx.save_for_backward(V64, pol)
        ctx.h, ctx.ws, ctx.k, ctx.gamma, ctx.b, ctx.seed, ctx.tol = h, ws, k, gamma, b, seed, tol
        ctx.dtypes = (c.dtype, val.dtype)
        ctx.stats = st
        return V64

    @staticmethod
    def backward(ctx, g):
        V64, pol = ctx.saved_tensors
        h = ctx.h
        n, m = h.n, h.m
        rp_t, col_t, val_t = mb.mdp_policy_transpose(h, pol, ctx.k, ctx.ws)
        g32 = g.detach().to(torch.float32).reshape(n, 1).contiguous()
        h_t = mb.mdp_create_csr(rp_t, col_t, val_t, g32, ctx.gamma)
        ws_t = mb.workspace(h_t, ctx.b)
        lam32 = torch.zeros(n, dtype=torch.float32, device=g.device)
        lam = torch.zeros(n, dtype=torch.float64, device=g.device)
        st = mb.vi_solve(h_t, lam32, ctx.b, ctx.seed, ws_t, tol_dv=ctx.tol, max_sweeps=1000000,
                         V64_out=lam)
        if not st["converged"]:
            raise RuntimeError("adjoint sweep did not converge: %s" % st)
        gc, gv = mb.mdp_value_gradients(h, pol, lam, V64, ctx.ws, k=ctx.k)
        ctx.adjoint_stats = st
        return (gc.view(n, m).to(ctx.dtypes[0]), gv.to(ctx.dtypes[1]), None, None, None, None,
                None, None, None)
