"""The allocation-free apply (hssx_apply_noalloc) against hssx_apply on the
same factors: two calls in a row, the second with a smaller input, both
precisions, both directions; sizes beyond the workspace are rejected."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_noalloc_apply_matches_apply():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    dev = torch.device("cuda:0")
    from paper_2105_07791_amd import hssx
    rng = np.random.default_rng(11)
    # first call: 129 x 129 grid, 6 right-hand sides; second: 33 x 33, 2
    for N, om, h_sw, nrhs, dtype in [(129, 32.0, 3, 6, "c128"), (33, 8.0, 1, 2, "c64")]:
        A = hssx.Operator(N, om, np.ones(N * N))
        P = hssx.Factor(A, tol=1e-6, leaf_size=32, beta=16, h_sw=h_sw, dtype=dtype, seed=1)
        assert P.stats()["n_hss_nodes"] > 0
        x = torch.tensor(rng.standard_normal((N * N, nrhs)) + 1j * rng.standard_normal((N * N, nrhs)),
                         device=dev)
        for trans in (False, True):
            y_ref = P.apply(x, trans=trans)
            y = P.apply_noalloc(x, trans=trans)
            err = (torch.linalg.vector_norm(y - y_ref) / torch.linalg.vector_norm(y_ref)).item()
            assert err <= 1e-13, (N, trans, err)


def test_noalloc_rejects_oversized_workspace():
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    from paper_2105_07791_amd import hssx
    from paper_2105_07791_amd._lib import HSSX_EINVAL, HssxError
    N = 257
    A = hssx.Operator(N, 50.0, np.ones(N * N))
    P = hssx.Factor(A, tol=1e-6, leaf_size=32, beta=16, h_sw=-1)
    x = torch.ones((N * N, 128), dtype=torch.complex128, device=dev)   # 2 n nrhs 16 B > 64 MiB
    with pytest.raises(HssxError) as e:
        P.apply_noalloc(x)
    assert e.value.code == HSSX_EINVAL
    y = P.apply_noalloc(x[:, :4].contiguous())      # a size that fits still works afterwards
    assert torch.isfinite(torch.view_as_real(y)).all()
