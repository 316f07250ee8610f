"""BF16 matrix-core convolution kernels of the learned warm start against the FP64
oracle.  Inputs are BF16-representable, so single layers differ from the oracle
only by FP32 accumulation order (outputs rounded to BF16 add 2^-9 relative);
whole-network gradients also carry the BF16 rounding of every activation."""
import numpy as np
import pytest

import gpu_setup as G
from oracle import cnn as ocnn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _built():
    G.ensure_built()


def _bf16(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16)


def _ctx():
    from paper_2608_06853_amd import _lib
    return _lib.Context(0)


@pytest.mark.parametrize("ci,co,st", [(2, 32, 1), (32, 32, 2), (32, 32, 1), (32, 1, 1), (16, 24, 2)])
def test_single_layer(ci, co, st):
    import torch
    rng = np.random.default_rng(ci * 100 + co + st)
    B, H, W = 2, 13, 10
    ctx = _ctx()
    x = _bf16(rng.standard_normal((B, H, W, ci)))
    w32 = rng.standard_normal((co, 9 * ci)).astype(np.float32) * 0.3
    wq = _bf16(w32).float().numpy().reshape(co, 3, 3, ci).astype(np.float64)
    b = rng.standard_normal(co).astype(np.float32)
    kp, ktp = ctx.conv_shapes(ci, co)
    wp = torch.empty(32 * kp, device="cuda", dtype=torch.bfloat16)
    wtp = torch.empty(32 * ktp, device="cuda", dtype=torch.bfloat16)
    ctx.conv3x3_pack(ci, co, torch.from_numpy(w32).cuda(), wp, wtp)
    Ho, Wo = (H - 1) // st + 1, (W - 1) // st + 1
    outf = torch.empty(B * Ho * Wo * co, device="cuda")
    xd = x.cuda().contiguous()
    ctx.conv3x3_fwd(B, H, W, ci, co, st, False, xd.view(-1), wp, torch.from_numpy(b).cuda(), outf=outf)
    xo = x.float().numpy().astype(np.float64)
    ref = ocnn.conv3x3(xo, wq, b.astype(np.float64), st)
    e = G.rel(outf.cpu().numpy().reshape(ref.shape), ref)
    print("fwd", ci, co, st, e, flush=True)
    assert e < 1e-5
    # backward data (with the ReLU mask of a random layer below) and weight
    dout = _bf16(rng.standard_normal((B, Ho, Wo, co)))
    act = _bf16(rng.standard_normal((B, H, W, ci)))
    din = torch.empty(B * H * W * ci, device="cuda", dtype=torch.bfloat16)
    ctx.conv3x3_bwd_data(B, H, W, ci, co, st, dout.cuda().view(-1), wtp, act.cuda().view(-1), din)
    dw = torch.empty(co * 9 * ci, device="cuda")
    db = torch.empty(co, device="cuda")
    ctx.conv3x3_bwd_weight(B, H, W, ci, co, st, xd.view(-1), dout.cuda().view(-1), dw, db)
    do = dout.float().numpy().astype(np.float64)
    dx, dwo, dbo = ocnn.conv3x3_backward(xo, wq, st, do)
    dx = dx * (act.float().numpy() > 0)
    e_dx = G.rel(din.float().cpu().numpy().reshape(dx.shape), dx)
    e_dw = G.rel(dw.cpu().numpy().reshape(dwo.shape), dwo)
    e_db = G.rel(db.cpu().numpy(), dbo)
    print("bwd", e_dx, e_dw, e_db, flush=True)
    assert e_dx < 4e-3 and e_dw < 1e-5 and e_db < 1e-5


@pytest.mark.parametrize("ci,co,st,B,H,W", [
    (32, 32, 2, 3, 70, 45),    # nine weight tiles: each wave owns tiles; many chunks per workgroup
    (8, 16, 1, 2, 33, 40),     # three tiles (Kp 80): the waves split the K-steps
    (4, 8, 2, 2, 50, 37),      # two tiles, element-wise input staging
    (2, 32, 1, 4, 64, 64),     # the first layer's shape
    (32, 1, 1, 3, 40, 41),     # one output channel, ragged last chunk
])
def test_weight_gradient_many_chunks(ci, co, st, B, H, W):
    """Weight and bias gradients over many 64-pixel chunks per workgroup, with a
    ragged tail, against the oracle."""
    import torch
    rng = np.random.default_rng(ci * 1000 + co * 10 + st)
    ctx = _ctx()
    Ho, Wo = (H - 1) // st + 1, (W - 1) // st + 1
    x = _bf16(rng.standard_normal((B, H, W, ci)))
    dout = _bf16(rng.standard_normal((B, Ho, Wo, co)))
    dw = torch.empty(co * 9 * ci, device="cuda")
    db = torch.empty(co, device="cuda")
    ctx.conv3x3_bwd_weight(B, H, W, ci, co, st, x.cuda().contiguous().view(-1),
                           dout.cuda().contiguous().view(-1), dw, db)
    w0 = np.zeros((co, 3, 3, ci))
    _, dwo, dbo = ocnn.conv3x3_backward(x.float().numpy().astype(np.float64), w0, st,
                                        dout.float().numpy().astype(np.float64))
    e_dw = G.rel(dw.cpu().numpy().reshape(dwo.shape), dwo)
    e_db = G.rel(db.cpu().numpy(), dbo)
    print("dw", ci, co, st, B, H, W, e_dw, e_db, flush=True)
    assert e_dw < 1e-5 and e_db < 1e-5


def test_network_gradients_match_oracle():
    import torch
    from paper_2608_06853_amd import cnn
    ctx = _ctx()
    net = cnn.WarmStartNet(ctx, seed=3)
    rng = np.random.default_rng(5)
    B = 2
    x = _bf16(rng.standard_normal((B, 128, 128, 2)))
    label = rng.standard_normal((B, 32, 32)).astype(np.float32)
    net.forward(x.cuda().contiguous().view(-1), B)
    loss = float(net.loss(torch.from_numpy(label).cuda(), B).item())
    net.backward(B)
    params = []
    for i, (ci, co, st, relu) in enumerate(ocnn.LAYERS):
        wq = _bf16(net.w[i].cpu().numpy()).float().numpy().reshape(co, 3, 3, ci).astype(np.float64)
        params.append((wq, net.b[i].cpu().numpy().astype(np.float64)))
    out, acts = ocnn.forward(params, x.float().numpy().astype(np.float64))
    lo, dout = ocnn.mse(out, label.reshape(B, 32, 32, 1).astype(np.float64), 1.0 / (B * 32 * 32))
    grads = ocnn.backward(params, acts, dout)
    print("loss", loss, lo, flush=True)
    assert abs(loss - lo) < 1e-2 * abs(lo)
    n = len(ocnn.LAYERS)
    for i in range(n):
        ew = G.rel(net.grads[i].cpu().numpy().reshape(grads[i][0].shape), grads[i][0])
        eb = G.rel(net.grads[n + i].cpu().numpy(), grads[i][1])
        print("layer", i, "dw", ew, "db", eb, flush=True)
        assert ew < 3e-2 and eb < 3e-2


def test_training_fits_a_batch():
    import torch
    from paper_2608_06853_amd import cnn
    ctx = _ctx()
    net = cnn.WarmStartNet(ctx, seed=1)
    rng = np.random.default_rng(7)
    B = 4
    x = _bf16(rng.standard_normal((B, 128, 128, 2))).cuda().contiguous().view(-1)
    y = torch.from_numpy(rng.standard_normal((B, 32, 32)).astype(np.float32) * 0.5).cuda()
    losses = [float(net.train_step(x, y, B, 3e-3).item()) for _ in range(150)]
    print("loss first/last", losses[0], losses[-1], flush=True)
    assert losses[-1] < 0.2 * losses[0]


@pytest.mark.parametrize("ci,co,st,B,H,W", [
    (3, 5, 2, 1, 1, 1),        # one pixel, odd channel counts (element-wise paths)
    (1, 1, 1, 1, 1, 2),        # one input and one output channel
    (12, 4, 2, 3, 2, 3),       # Cin not a multiple of 8, Cout a multiple of 4 (8-byte stores)
    (8, 16, 2, 2, 3, 1),       # stride-2 input gradient by parity class; two classes empty
    (32, 32, 2, 1, 5, 7),      # the same with two K-steps per tap, odd height and width
    (2, 8, 1, 3, 9, 11),       # the two-channel forward operand of the first layer
])
def test_degenerate_shapes(ci, co, st, B, H, W):
    """Forward, input gradient and weight gradient at sizes below one tile."""
    import torch
    rng = np.random.default_rng(ci * 7 + co * 3 + st + H)
    ctx = _ctx()
    Ho, Wo = (H - 1) // st + 1, (W - 1) // st + 1
    x = _bf16(rng.standard_normal((B, H, W, ci)))
    w32 = rng.standard_normal((co, 9 * ci)).astype(np.float32) * 0.3
    wq = _bf16(w32).float().numpy().reshape(co, 3, 3, ci).astype(np.float64)
    b = rng.standard_normal(co).astype(np.float32)
    kp, ktp = ctx.conv_shapes(ci, co)
    wp = torch.empty(32 * kp, device="cuda", dtype=torch.bfloat16)
    wtp = torch.empty(32 * ktp, device="cuda", dtype=torch.bfloat16)
    ctx.conv3x3_pack(ci, co, torch.from_numpy(w32).cuda(), wp, wtp)
    xd = x.cuda().contiguous().view(-1)
    outf = torch.empty(B * Ho * Wo * co, device="cuda")
    ctx.conv3x3_fwd(B, H, W, ci, co, st, False, xd, wp, torch.from_numpy(b).cuda(), outf=outf)
    xo = x.float().numpy().astype(np.float64)
    ref = ocnn.conv3x3(xo, wq, b.astype(np.float64), st)
    assert G.rel(outf.cpu().numpy().reshape(ref.shape), ref) < 1e-5
    dout = _bf16(rng.standard_normal((B, Ho, Wo, co)))
    din = torch.empty(B * H * W * ci, device="cuda", dtype=torch.bfloat16)
    ctx.conv3x3_bwd_data(B, H, W, ci, co, st, dout.cuda().contiguous().view(-1), wtp, None, din)
    dw = torch.empty(co * 9 * ci, device="cuda")
    db = torch.empty(co, device="cuda")
    ctx.conv3x3_bwd_weight(B, H, W, ci, co, st, xd, dout.cuda().contiguous().view(-1), dw, db)
    dx, dwo, dbo = ocnn.conv3x3_backward(xo, wq, st, dout.float().numpy().astype(np.float64))
    e = (G.rel(din.float().cpu().numpy().reshape(dx.shape), dx),
         G.rel(dw.cpu().numpy().reshape(dwo.shape), dwo), G.rel(db.cpu().numpy(), dbo))
    print("degenerate", ci, co, st, B, H, W, e, flush=True)
    assert e[0] < 4e-3 and e[1] < 1e-5 and e[2] < 1e-5


def test_features_match_oracle():
    """Network input: (map - shift) * scale in FP32, rounded to BF16 to nearest
    even, against the FP64 value rounded by the oracle.  The two can differ by one
    BF16 step only where the FP64 value lies within FP32 rounding of a tie."""
    import torch
    ctx = _ctx()
    rng = np.random.default_rng(7)
    C, n = 2, 128 * 128 + 37
    maps = rng.standard_normal((C, n)).astype(np.float32)
    shift = np.array([0.6, 0.3], np.float32)
    scale = np.array([2.0, 3.0], np.float32)
    out = torch.empty(n * C, device="cuda", dtype=torch.bfloat16)
    ctx.features(torch.from_numpy(maps.ravel()).cuda(), torch.from_numpy(shift).cuda(),
                 torch.from_numpy(scale).cuda(), out)
    got = out.float().cpu().numpy().astype(np.float64).reshape(n, C)
    exact = ocnn.features(maps, shift.astype(np.float64), scale.astype(np.float64))
    want = ocnn.bf16_round(exact)
    differ = got != want
    # where they differ, the exact value is a BF16 tie up to FP32 rounding
    lo = np.minimum(got, want)
    hi = np.maximum(got, want)
    tie = np.abs(exact - 0.5 * (lo + hi)) <= 4e-7 * np.abs(exact)
    print("features: entries", got.size, "differing", int(differ.sum()), flush=True)
    assert np.all(tie[differ])
    assert differ.mean() < 1e-3


@pytest.mark.parametrize("clamp", [False, True])
def test_polar_to_grid_matches_oracle(clamp):
    """Output resampling of the network: slowness on the node grid from the polar
    map (bilinear, clamped to the map), against the oracle at every node."""
    import torch
    ctx = _ctx()
    rng = np.random.default_rng(11)
    nr, nt = 32, 32
    pmap = rng.standard_normal((nr, nt)).astype(np.float32)
    r0, dr, t0, dt = 41.5, 1.8, -0.15, 0.0095
    nx, nz, x0, z0, dx, dz = 37, 29, -22.0, 36.0, 1.3, 2.4      # reaches past the map
    s_lo, s_hi = (0.62, 0.68) if clamp else (0.1, 10.0)
    out = torch.empty(nz * nx, device="cuda")
    ctx.polar_to_grid(torch.from_numpy(pmap.ravel()).cuda(), nr, nt, r0, dr, t0, dt, nx, nz, x0,
                      z0, dx, dz, 1.0 / 1.54, 0.03, s_lo, s_hi, out)
    got = out.cpu().numpy().reshape(nz, nx).astype(np.float64)
    want = ocnn.polar_to_grid(pmap, r0, dr, t0, dt, nx, nz, x0, z0, dx, dz, 1.0 / 1.54, 0.03,
                              s_lo, s_hi)
    err = np.max(np.abs(got - want) / np.abs(want))
    print("polar_to_grid max rel err", err, "clamped nodes",
          int(np.sum((want == s_lo) | (want == s_hi))), flush=True)
    assert err < 1e-5
