"""The feature pass without a scratch argument (mmas_mlp_features_noalloc,
for callers that cannot allocate): its outputs equal those of
mmas_mlp_features bit for bit on two calls in a row, the second on a smaller
instance (the static scratch keeps the first call's contents), and sizes
beyond the static scratch are refused before any HIP call."""
import numpy as np
import pytest

from paper_2003_11902_amd import instances as I


def test_refuses_sizes_beyond_the_static_scratch():
    from paper_2003_11902_amd import mmas as M
    # arguments are checked before any device call, so this runs without a GPU
    one = np.zeros(1, dtype=np.int64)
    ptr = one.ctypes.data
    assert M.lib.mmas_mlp_features_noalloc(ptr, ptr, 65536, ptr, None, ptr, None) == M.MMAS_EINVAL
    assert M.lib.mmas_mlp_features_noalloc(ptr, ptr, 16, ptr, None, ptr, None) == M.MMAS_EINVAL
    assert M.lib.mmas_mlp_features_noalloc(None, ptr, 100, ptr, None, ptr, None) == M.MMAS_EINVAL


@pytest.mark.gpu
def test_equals_the_scratch_argument_form_on_two_calls():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_11902_amd import mmas as M
    for kind, n, seed in (("clustered", 900, 41), ("uniform", 257, 42)):
        print(f"no-alloc features: {kind} n = {n} seed {seed}", flush=True)
        xy, d = I.make_instance(kind, n, seed=seed)
        dist = torch.from_numpy(d).cuda()
        xyt = torch.from_numpy(xy.astype(np.float32)).cuda()
        knn_a, X_a, f_a = M.mmas_mlp_features_noalloc(dist, xyt, with_features=True)
        knn_b, X_b, f_b = M.mmas_mlp_features(dist, xyt, with_features=True)
        torch.cuda.synchronize()
        assert torch.equal(knn_a, knn_b)
        assert torch.equal(X_a, X_b)
        assert np.array_equal(f_a.cpu().numpy().view(np.uint32), f_b.cpu().numpy().view(np.uint32))
