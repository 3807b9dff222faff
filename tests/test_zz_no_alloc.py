"""dg_mlp_infer_noalloc (the network's FP32 forward with its activations in
the library's fixed device array) against dg_mlp_infer's FP32 path, which
allocates its workspace: the same kernels, so the outputs must agree bit for
bit, on two calls in a row (the second with fewer rows, over what the first
left in the array), and both against the FP64 oracle forward.  Rows beyond the
array's capacity are rejected without touching the device."""
import numpy as np
import pytest

import paper_1710_03887_amd as dg
from oracle import mlp as omlp
from workloads.mlp_init import init_params

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _rows(B, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(scale=0.5, size=(B, 78))
    n = rng.normal(size=(B, 3))
    X[:, 75:] = n / np.linalg.norm(n, axis=1, keepdims=True)
    return X.astype(np.float32)


def test_noalloc_matches_allocating_forward():
    p = init_params(3).astype(np.float32)
    m = dg.dg_mlp_create(p)
    cap = dg.DG_MLP_NOALLOC_ROWS
    # a full array first, then a smaller, ragged row count over its leftovers
    for B, seed in ((cap, 11), (1000 + 13, 12)):
        X = _rows(B, seed)
        print(f"noalloc forward: B = {B}, seed {seed}", flush=True)
        Xd = torch.from_numpy(X).cuda()
        Y_ref = torch.full((B, 75), np.nan, dtype=torch.float32, device="cuda")
        Y_na = torch.full((B, 75), np.nan, dtype=torch.float32, device="cuda")
        dg.dg_mlp_infer(m, Xd, Y_ref, bf16=False)
        dg.dg_mlp_infer_noalloc(m, Xd, Y_na)
        torch.cuda.synchronize()
        a, b = Y_ref.cpu().numpy(), Y_na.cpu().numpy()
        assert np.isfinite(b).all()
        assert np.array_equal(a, b), f"max |diff| {np.abs(a - b).max():.3e}"
        Y_or, _ = omlp.forward(p.astype(np.float64), X.astype(np.float64))
        err = np.abs(b - Y_or).max() / np.abs(Y_or).max()
        print(f"  bitwise equal to dg_mlp_infer; max rel err vs oracle {err:.2e}")
        assert err < 1e-5
    # capacity: rejected with a clear error, nothing launched
    X = torch.zeros((cap + 1, 78), dtype=torch.float32, device="cuda")
    Y = torch.zeros((cap + 1, 75), dtype=torch.float32, device="cuda")
    with pytest.raises(dg.DGError, match="DG_MLP_NOALLOC_ROWS"):
        dg.dg_mlp_infer_noalloc(m, X, Y)
    # no rows: nothing to do
    dg.dg_mlp_infer_noalloc(m, X[:0], Y[:0])
    dg.dg_mlp_destroy(m)
