"""GPU tests of the surface-flux surrogate kernels through the C ABI.

The network is not part of the paper, so its parity is pinned by the CPU
network oracle (FP64 sums, BF16 rounding emulated at the points where the
kernels store BF16) and by its own gradient check, not by the paper.

Tolerances.  The kernels accumulate in FP32 and store hidden activations and
gradients in BF16.  Against the oracle with the same BF16 rounding points,
the differences come from the summation order and FP32 accumulation
(relative ~sqrt(K) 2^-24 per dot product).  Now and then that moves a value
across a BF16 rounding boundary -- a change of one BF16 ulp (2^-8 relative)
in that element, with probability ~sqrt(K) 2^-24 / 2^-9 ~ 3e-4 per element
at K = 512 -- and each such flip reaches an output or gradient diluted over
the fan-in (~2^-8 / sqrt(512) ~ 2e-4 relative per flip), compounding over
the layers a gradient passes through (up to 2 x depth + 1 BF16 stores).
Relative L2 errors are bounded by 3e-3 here, and where the batch resolves it
the error must also stay below 0.3 x the BF16-vs-FP64 difference (the oracle
without BF16 rounding): the kernels round where the oracle says.
"""
import ctypes as C
import math

import numpy as np
import pytest

from oracle import mlp_ref
from paper_1703_10119_amd import dfhm, workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _bf16_bits(x):
    """BF16 bit patterns (RNE) of an array, as int16 for a torch tensor."""
    f = np.ascontiguousarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    return u.view(np.int16)


def _bits_to_f(b):
    return (np.asarray(b).view(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _net(dims, batch, seed=3, wd=0.0, pairs=False):
    from paper_1703_10119_amd import surrogate
    n_in, width, depth, n_out = dims
    return surrogate.MLP(n_in=n_in, width=width, depth=depth, n_out=n_out, max_batch=batch,
                         seed=seed, weight_decay=wd, act_pairs=pairs)


# ragged against the 128 x 128 x 32 tiles in every dimension
DIMS = [(40, 136, 2, 4), (584, 512, 4, 8), (8, 8, 1, 4)]
BATCH = [300, 1000, 1]


@pytest.mark.parametrize("pairs", [False, True])
@pytest.mark.parametrize("dims,batch", list(zip(DIMS, BATCH)))
def test_forward_matches_oracle(dims, batch, pairs):
    dev = _dev()
    rng = np.random.default_rng(11)
    theta = mlp_ref.init(*dims[:3], seed=5, n_out=dims[3])
    theta[-dims[3]:] = rng.normal(0, 0.2, dims[3])
    x = rng.normal(0, 1, (batch, dims[0]))
    xb = _bf16_bits(x)
    net = _net(dims, batch, pairs=pairs)
    net.set_params(theta)
    y = net.forward(torch.tensor(xb, device=dev)).cpu().numpy().astype(np.float64)
    ref, _ = mlp_ref.forward(theta, _bits_to_f(xb), dims, bf=True, pairs=pairs)
    ref_fp64, _ = mlp_ref.forward(theta, x, dims, bf=False)
    e = _rel(y, ref)
    print(f"forward dims={dims} batch={batch} pairs={pairs}: rel L2 vs bf16 oracle {e:.2e}, "
          f"bf16 oracle vs fp64 {_rel(ref, ref_fp64):.2e}")
    assert e <= 3e-3
    if batch >= 100:
        assert e < 0.2 * _rel(ref, ref_fp64)
    net.close()


@pytest.mark.parametrize("pairs", [False, True])
@pytest.mark.parametrize("dims,batch", list(zip(DIMS, BATCH)))
def test_gradients_match_oracle(dims, batch, pairs):
    dev = _dev()
    rng = np.random.default_rng(12)
    F = dims[3] // 2
    theta = mlp_ref.init(*dims[:3], seed=6, n_out=dims[3])
    theta[-dims[3]:] = rng.normal(0, 0.2, dims[3])
    x = rng.normal(0, 1, (batch, dims[0]))
    y = rng.normal(0, 1, (batch, F))
    xb = _bf16_bits(x)
    net = _net(dims, batch, pairs=pairs)
    net.set_params(theta)
    g, loss = net.gradients(torch.tensor(xb, device=dev),
                            torch.tensor(y, dtype=torch.float32, device=dev))
    y32 = y.astype(np.float32).astype(np.float64)
    rl, rg = mlp_ref.loss_and_grad(theta, _bits_to_f(xb), y32, dims, bf=True, pairs=pairs)
    _, rg64 = mlp_ref.loss_and_grad(theta, x, y32, dims, bf=False)
    # the loss moves with the outputs (rel L2 <= 3e-3 above): 1e-3 relative
    assert abs(loss - rl) <= 1e-3 * max(1.0, abs(rl))
    # per layer (weights and biases separately)
    o = 0
    for n, k in mlp_ref.shapes(*dims[:3], n_out=dims[3]):
        for size in (n * k, n):
            e = _rel(g[o:o + size].astype(np.float64), rg[o:o + size])
            gap = _rel(rg[o:o + size], rg64[o:o + size])
            print(f"grad block @{o} size {size}: rel L2 {e:.2e} (bf16 vs fp64 {gap:.2e})")
            assert e <= 3e-3, (o, size, e)
            if batch >= 100:
                assert e < 0.3 * gap, (o, size, e, gap)
            o += size
    assert o == g.size
    net.close()


def test_adamw_first_step():
    """First AdamW step: m_hat = g, v_hat = g^2, so w' = w - lr (g/(|g|+eps) + wd w)."""
    dev = _dev()
    dims, batch = (24, 64, 2, 4), 200
    rng = np.random.default_rng(13)
    theta = mlp_ref.init(*dims[:3], seed=7)
    x = torch.tensor(_bf16_bits(rng.normal(0, 1, (batch, dims[0]))), device=dev)
    y = torch.tensor(rng.normal(0, 1, (batch, 2)), dtype=torch.float32, device=dev)
    lr, wd = 1e-3, 0.01
    net = _net(dims, batch, wd=wd)
    net.set_params(theta)
    g, _ = net.gradients(x, y)
    net.train_step(x, y, lr)
    w1 = net.get_params().astype(np.float64)
    t32 = theta.astype(np.float32).astype(np.float64)
    g = g.astype(np.float64)
    want = t32 - lr * (g / (np.abs(g) + 1e-8) + wd * t32)
    assert np.max(np.abs(w1 - want)) <= 1e-6 * lr + 1e-7 * np.abs(t32).max()
    net.close()


def test_training_reduces_loss():
    """A smooth target the network can fit: the loss falls several-fold."""
    dev = _dev()
    dims, batch = (64, 256, 3, 4), 4096
    rng = np.random.default_rng(14)
    X = rng.normal(0, 1, (batch * 4, dims[0]))
    Y = np.stack([np.tanh(X[:, :8].sum(1) / 3), np.sin(X[:, 8:16].mean(1) * 2)], 1)
    Xd = torch.tensor(_bf16_bits(X), device=dev)
    Yd = torch.tensor(Y, dtype=torch.float32, device=dev)
    net = _net(dims, batch, seed=9)
    losses = []
    for it in range(400):
        b = it % 4
        l = net.train_step(Xd[b * batch:(b + 1) * batch], Yd[b * batch:(b + 1) * batch], 2e-3,
                           want_loss=(it % 50 == 0 or it == 399))
        if l is not None:
            losses.append(l)
    print("losses", losses)
    assert all(math.isfinite(v) for v in losses)
    # loss = MSE + variance terms; a fitted network drives both down
    assert losses[-1] < losses[0] - 2.0
    net.close()


def test_features_match_definition():
    """Feature rows against the header's definition, evaluated in numpy with
    the same FP64 sinusoid and FP32 normalisation."""
    dev = _dev()
    from paper_1703_10119_amd import surrogate as S
    walls = wl.uniform_batch(5, seed=21, nx=51)
    sines, params = S.wall_inputs(walls)
    rng = np.random.default_rng(15)
    n = 37
    wall_of = rng.integers(0, 5, n).astype(np.int32)
    t = rng.uniform(48 * 3600, 80 * 3600, n)
    desc = S.feature_desc(params, 48 * 3600, 80 * 3600)
    x = S.features(torch.tensor(wall_of, device=dev), torch.tensor(t, device=dev),
                   torch.tensor(sines, device=dev), torch.tensor(params, device=dev), desc)
    got = _bits_to_f(x.cpu().numpy())
    H = S.N_HIST
    want = np.zeros((n, S.STRIDE))
    for s in range(n):
        w, ts = wall_of[s], t[s] - (H - 1 - np.arange(H)) * 600.0
        Tv = (sines[w, 0] + sines[w, 1] * np.sin(2 * np.pi * ts / sines[w, 2] + sines[w, 3])).astype(np.float32)
        Rv = (sines[w, 4] + sines[w, 5] * np.sin(2 * np.pi * ts / sines[w, 6] + sines[w, 7])).astype(np.float32)
        want[s, :H] = (Tv - np.float32(desc.T_mean)) / np.float32(desc.T_scale)
        want[s, H:2 * H] = (Rv - np.float32(desc.RH_mean)) / np.float32(desc.RH_scale)
        ph = 2 * np.pi * np.fmod(t[s], 86400.0) / 86400.0
        raw = np.concatenate([params[w], np.float32([t[s] / 86400.0, np.sin(ph), np.cos(ph)])])
        pm = np.array(desc.p_mean[:], np.float32)
        ps = np.array(desc.p_scale[:], np.float32)
        want[s, 2 * H:2 * H + 8] = (raw.astype(np.float32) - pm) / ps
    want = mlp_ref.bf16(want)
    ulp = np.maximum(np.abs(want), 1e-30) * 2.0 ** -7
    assert np.all(np.abs(got - want) <= ulp + 1e-30)
    assert np.mean(got == want) > 0.999


def test_decode_and_fallback_flags():
    """Decode against its definition: flux = u exp(l) with u, l de-normalised,
    fallback when sd(u) + |u| sd(l) > tau for either field."""
    dev = _dev()
    rng = np.random.default_rng(16)
    B = 1000
    y = rng.normal(0, 1, (B, 8)).astype(np.float32)
    y[:, 4:] = rng.uniform(-20, -4, (B, 4))
    scale = np.array([0.1, 1.2, -0.3, 0.9, 1.0, 0.5, -14.0, 0.8], np.float32)
    tau = 0.01
    flux = torch.empty((B, 2), dtype=torch.float32, device=dev)
    fb = torch.empty(B, dtype=torch.uint8, device=dev)
    yd = torch.tensor(y, device=dev)
    st = dfhm.load().dfhm_mlp_decode(yd.data_ptr(), B, scale.ctypes.data_as(C.c_void_p), tau,
                                     flux.data_ptr(), fb.data_ptr(),
                                     torch.cuda.current_stream().cuda_stream)
    assert st == 0
    torch.cuda.synchronize()
    m, sd = scale[0::2].astype(np.float64), scale[1::2].astype(np.float64)
    yv = y.astype(np.float64)
    u = yv[:, :2] * sd[:2] + m[:2]
    lg = yv[:, 2:4] * sd[2:] + m[2:]
    want = u * np.exp(lg)
    f = flux.cpu().numpy().astype(np.float64)
    # FP32: u = y std + mean may cancel, so its error is relative to |y std| + |mean|
    bound = 1e-6 * (np.abs(yv[:, :2] * sd[:2]) + np.abs(m[:2])) * np.exp(lg) + 1e-5 * np.abs(want)
    assert np.all(np.abs(f - want) <= bound)
    e = sd[:2] * np.exp(0.5 * yv[:, 4:6]) + np.abs(u) * sd[2:] * np.exp(0.5 * yv[:, 6:8])
    flag = np.any(e > tau, axis=1)
    clear = np.all(np.abs(e / tau - 1) > 1e-4, axis=1)
    got = fb.cpu().numpy().astype(bool)
    assert 0.05 < flag.mean() < 0.95
    assert np.array_equal(got[clear], flag[clear])
    bad = scale.copy()
    bad[1] = 0.0
    assert dfhm.load().dfhm_mlp_decode(yd.data_ptr(), B, bad.ctypes.data_as(C.c_void_p), tau,
                                       flux.data_ptr(), fb.data_ptr(), None) == 1


def test_decode_ensemble_is_the_member_mean():
    """Ensemble decode against its definition: flux and predicted error are
    the means of the members' values; one member gives dfhm_mlp_decode's
    results bit for bit; bad member counts or a null member are refused."""
    dev = _dev()
    rng = np.random.default_rng(17)
    B, K = 777, 3
    ys = []
    for _ in range(K):
        y = rng.normal(0, 1, (B, 8)).astype(np.float32)
        y[:, 4:] = rng.uniform(-20, -4, (B, 4))
        ys.append(y)
    scale = np.array([0.1, 1.2, -0.3, 0.9, 1.0, 0.5, -14.0, 0.8], np.float32)
    tau = 0.01
    L = dfhm.load()
    st_ = torch.cuda.current_stream().cuda_stream
    yd = [torch.tensor(y, device=dev) for y in ys]
    ptrs = (C.c_void_p * K)(*[t.data_ptr() for t in yd])
    flux = torch.empty((B, 2), dtype=torch.float32, device=dev)
    fb = torch.empty(B, dtype=torch.uint8, device=dev)
    assert L.dfhm_mlp_decode_ensemble(ptrs, K, B, scale.ctypes.data_as(C.c_void_p), tau,
                                      flux.data_ptr(), fb.data_ptr(), st_) == 0
    torch.cuda.synchronize()
    m, sd = scale[0::2].astype(np.float64), scale[1::2].astype(np.float64)
    want = np.zeros((B, 2))
    e = np.zeros((B, 2))
    bound = np.zeros((B, 2))
    for y in ys:
        yv = y.astype(np.float64)
        u = yv[:, :2] * sd[:2] + m[:2]
        lg = yv[:, 2:4] * sd[2:] + m[2:]
        want += u * np.exp(lg) / K
        e += (sd[:2] * np.exp(0.5 * yv[:, 4:6]) + np.abs(u) * sd[2:] * np.exp(0.5 * yv[:, 6:8])) / K
        bound += (1e-6 * (np.abs(yv[:, :2] * sd[:2]) + np.abs(m[:2])) * np.exp(lg)
                  + 1e-5 * np.abs(u * np.exp(lg))) / K
    f = flux.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(f - want) <= bound + 1e-6 * np.abs(want))
    flag = np.any(e > tau, axis=1)
    clear = np.all(np.abs(e / tau - 1) > 1e-4, axis=1)
    got = fb.cpu().numpy().astype(bool)
    assert 0.05 < flag.mean() < 0.95
    assert np.array_equal(got[clear], flag[clear])
    # one member = dfhm_mlp_decode, bit for bit
    one = (C.c_void_p * 1)(yd[1].data_ptr())
    f1 = torch.empty((B, 2), dtype=torch.float32, device=dev)
    b1 = torch.empty(B, dtype=torch.uint8, device=dev)
    f2 = torch.empty((B, 2), dtype=torch.float32, device=dev)
    b2 = torch.empty(B, dtype=torch.uint8, device=dev)
    assert L.dfhm_mlp_decode_ensemble(one, 1, B, scale.ctypes.data_as(C.c_void_p), tau,
                                      f1.data_ptr(), b1.data_ptr(), st_) == 0
    assert L.dfhm_mlp_decode(yd[1].data_ptr(), B, scale.ctypes.data_as(C.c_void_p), tau,
                             f2.data_ptr(), b2.data_ptr(), st_) == 0
    torch.cuda.synchronize()
    assert torch.equal(f1, f2) and torch.equal(b1, b2)
    for n in (0, 5):
        assert L.dfhm_mlp_decode_ensemble(ptrs, n, B, scale.ctypes.data_as(C.c_void_p), tau,
                                          flux.data_ptr(), fb.data_ptr(), st_) == 1
    holed = (C.c_void_p * 2)(yd[0].data_ptr(), None)
    assert L.dfhm_mlp_decode_ensemble(holed, 2, B, scale.ctypes.data_as(C.c_void_p), tau,
                                      flux.data_ptr(), fb.data_ptr(), st_) == 1
    assert L.dfhm_mlp_decode_ensemble(None, 2, B, scale.ctypes.data_as(C.c_void_p), tau,
                                      flux.data_ptr(), fb.data_ptr(), st_) == 1


def test_mlp_argument_errors():
    _dev()
    from paper_1703_10119_amd import surrogate as S
    L = dfhm.load()
    h = C.c_void_p()
    for bad in [dict(n_in=12), dict(width=0), dict(depth=17), dict(n_out=33), dict(max_batch=0)]:
        kw = dict(n_in=16, width=16, depth=1, n_out=4, max_batch=8)
        kw.update(bad)
        c = dfhm.MlpConfig(kw["n_in"], kw["width"], kw["depth"], kw["n_out"], kw["max_batch"], 0,
                           0, 0.9, 0.999, 1e-8, 0.0, None)
        assert L.dfhm_mlp_create(C.byref(c), C.byref(h)) == 1, bad     # DFHM_E_INVAL
    net = S.MLP(n_in=16, width=16, depth=1, n_out=4, max_batch=8)
    x = torch.zeros((9, 16), dtype=torch.int16, device="cuda")
    with pytest.raises(dfhm.DfhmError):
        net.forward(x)                                    # batch above max_batch
    net.close()
