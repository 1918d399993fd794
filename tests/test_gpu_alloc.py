"""The boundary's allocator injection: handles created under a context take
every device buffer from the caller's allocator (here torch's caching
allocator) and give every byte back; results equal those of the library's
own allocations."""
import gc

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from synth import make_problem  # noqa: E402


def test_context_allocator_sees_every_byte_returned():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    dev = torch.device("cuda:0")
    from paper_2105_07791_amd import hssx
    N, om = 65, 16.0
    pr = make_problem("helmholtz_p1_65", N=N, omega=om, seed=3, nsrc=3)
    s = np.ones(N * N)
    f = torch.tensor(pr.f, device=dev)
    kw = dict(tol=1e-6, leaf_size=32, beta=16, h_sw=2, dtype="c64", seed=1)
    A0 = hssx.Operator(N, om, s)
    P0 = hssx.Factor(A0, **kw)
    b0 = A0.load(f)
    x0, _ = hssx.gmres_solve(A0, P0, b0, flexible=True)
    ctx = hssx.Context(0)
    with ctx:
        A = hssx.Operator(N, om, s)
        P = hssx.Factor(A, **kw)
    # later calls on the context's handles still allocate through it
    b = A.load(f)
    x, st = hssx.gmres_solve(A, P, b, flexible=True)
    P.refactor(A)
    y = P.apply(b)
    y0 = P0.apply(b0)
    live = ctx.stats()
    assert live["allocs"] > 0 and live["live_bytes"] > 0
    assert all(v["converged"] for v in st)
    assert torch.linalg.vector_norm(x - x0).item() <= 1e-13 * torch.linalg.vector_norm(x0).item()
    assert torch.linalg.vector_norm(y - y0).item() <= 1e-13 * torch.linalg.vector_norm(y0).item()
    del P, A, x, y
    gc.collect()
    torch.cuda.synchronize()
    ctx.destroy()
    assert ctx.alloc_calls > 0
    assert ctx.alloc_calls == ctx.free_calls, (ctx.alloc_calls, ctx.free_calls)
    assert ctx.alloc_bytes == ctx.free_bytes, (ctx.alloc_bytes, ctx.free_bytes)
