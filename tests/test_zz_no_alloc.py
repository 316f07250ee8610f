"""The no-allocation weight-gradient entry point (af_conv3x3_bwd_weight_noalloc,
partial sums in the library's static device array) against the allocating one
(af_conv3x3_bwd_weight): bit-identical results on two calls in a row, the second
with a smaller input (the array keeps the first call's contents), and both
against the FP64 oracle (1e-5).  It ends with the largest shape, so it also covers
a call that fills all of the array's workgroup slabs."""
import numpy as np
import pytest

import gpu_setup as G
from oracle import cnn as ocnn

pytestmark = pytest.mark.gpu


def _bf16(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16)


def _run(ctx, ci, co, st, B, H, W, seed):
    import torch
    rng = np.random.default_rng(seed)
    Ho, Wo = (H - 1) // st + 1, (W - 1) // st + 1
    x = _bf16(rng.standard_normal((B, H, W, ci)))
    dout = _bf16(rng.standard_normal((B, Ho, Wo, co)))
    xd, dd = x.cuda().view(-1), dout.cuda().view(-1)
    out = {}
    for noalloc in (True, False):
        dw = torch.full((co * 9 * ci,), float("nan"), device="cuda")
        db = torch.full((co,), float("nan"), device="cuda")
        ctx.conv3x3_bwd_weight(B, H, W, ci, co, st, xd, dd, dw, db, noalloc=noalloc)
        torch.cuda.synchronize()
        out[noalloc] = (dw.cpu().numpy(), db.cpu().numpy())
    xo = x.float().numpy().astype(np.float64)
    wq = np.zeros((co, 3, 3, ci))
    _, dwo, dbo = ocnn.conv3x3_backward(xo, wq, st, dout.float().numpy().astype(np.float64))
    return out, dwo, dbo


@pytest.mark.parametrize("seq", ["large_then_small", "small_then_largest"])
def test_noalloc_weight_gradient_matches_allocating_call(seq):
    G.ensure_built()
    from paper_2608_06853_amd import _lib
    ctx = _lib.Context(0)
    shapes = {"large_then_small": [(32, 32, 1, 4, 64, 64), (2, 32, 2, 2, 13, 10)],
              "small_then_largest": [(4, 8, 2, 2, 50, 37), (32, 32, 1, 16, 128, 128)]}[seq]
    for k, (ci, co, st, B, H, W) in enumerate(shapes):
        print("no-allocation weight gradient", seq, "call", k + 1, "shape", (ci, co, st, B, H, W),
              flush=True)
        out, dwo, dbo = _run(ctx, ci, co, st, B, H, W, seed=17 + k)
        (dw_n, db_n), (dw_a, db_a) = out[True], out[False]
        assert np.array_equal(dw_n, dw_a) and np.array_equal(db_n, db_a)
        assert np.all(np.isfinite(dw_n)) and np.all(np.isfinite(db_n))
        e_dw = G.rel(dw_n.reshape(dwo.shape), dwo)
        e_db = G.rel(db_n, dbo)
        print("  bit-identical to the allocating call; vs oracle dw", e_dw, "db", e_db, flush=True)
        assert e_dw < 1e-5 and e_db < 1e-5


def test_noalloc_rejects_bad_arguments():
    import torch
    G.ensure_built()
    from paper_2608_06853_amd import _lib
    ctx = _lib.Context(0)
    x = torch.zeros(4 * 4 * 33, device="cuda", dtype=torch.bfloat16)
    dw = torch.empty(32 * 9 * 33, device="cuda")
    db = torch.empty(32, device="cuda")
    with pytest.raises(_lib.AfError) as e:        # Cin above 32
        ctx.conv3x3_bwd_weight(1, 4, 4, 33, 32, 1, x, torch.zeros(4 * 4 * 32, device="cuda",
                                                                   dtype=torch.bfloat16),
                               dw, db, noalloc=True)
    assert e.value.status == _lib.AF_ERR_ARG
