"""GPU tests of the surface-flux surrogate kernels through the C ABI.

The network is not part of the paper, so its parity is pinned by the CPU
network oracle (FP64 sums, BF16 rounding at the points where the kernels
store BF16) and by its own gradient check, not by the paper.

Element by element, layer by layer.  Each layer is checked given the GPU's
own inputs to that layer (its stored BF16 activations, pre-activations and
gradients, read back through dfhm_mlp_get_intermediate), so that every
element has an exact FP64 value and a rigorous interval for the GPU result:
  * a K-term dot product of BF16 operands accumulated in FP32 in any order
    (the products are exact in FP32) is within gamma_K sum |a b| of the exact
    sum, gamma_K = K 2^-24 / (1 - K 2^-24); one more FP32 rounding per bias
    add or product;
  * GELU is 1.13-Lipschitz, and the FP32 GELU (erff) and its derivative are
    within 1e-6 |z| + 1e-7 of the exact ones;
  * BF16 rounding (nearest even) is monotone, so a BF16 value computed from
    anything inside [lo, hi] lies in [bf16(lo), bf16(hi)].
Every element must lie in its interval: activations, pre-activations,
outputs, every backpropagated gradient and every weight and bias gradient.
Across the whole network (no teacher forcing) a value now and then crosses a
BF16 rounding boundary on one side and not the other, a flip of one BF16 ulp
that then spreads through the following layers; there the relative L2 error
must stay below 3e-3 and below 0.3 x the gap between the BF16 and the FP64
oracle (the kernels round where the oracle says), and the test reports how
many outputs fall outside their no-flip interval.
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


def _net(dims, batch, seed=3, wd=0.0):
    from paper_1703_10119_amd import surrogate
    n_in, width, depth, n_out = dims
    return surrogate.MLP(n_in=n_in, width=width, depth=depth, n_out=n_out, max_batch=batch,
                         seed=seed, weight_decay=wd)


# ragged against the 128 x 128 x 32 tiles in every dimension
DIMS = [(40, 136, 2, 4), (584, 512, 4, 8), (8, 8, 1, 4)]
BATCH = [300, 1000, 1]

U32 = 2.0 ** -24


def _gamma(k):
    return k * U32 / (1.0 - k * U32)


def _bf(x):
    return mlp_ref.bf16(x)


def _gelu_exact(z):
    return mlp_ref.gelu(z)


def _in_bf16_interval(got, lo, hi):
    """got (BF16 values as FP64) within [bf16(lo), bf16(hi)], elementwise."""
    return (got >= _bf(lo)) & (got <= _bf(hi))


def _dot_interval(A, B, bias=None):
    """Exact A @ B (+ bias) in FP64 and the FP32 accumulation bound of each
    element (products exact, any summation order, one rounding for the bias
    add; a 2^-53 K term covers the FP64 reference sum itself)."""
    K = A.shape[1]
    s = A @ B
    mag = np.abs(A) @ np.abs(B)
    if bias is not None:
        s = s + bias
    bound = (_gamma(K + 1) + K * 2.0 ** -53) * mag + U32 * np.abs(s) + 1e-30
    return s, bound


def _layers(net, theta):
    return [(_bf(W), b.astype(np.float32).astype(np.float64))
            for W, b in mlp_ref.unpack(theta, *net.dims)]


@pytest.mark.parametrize("dims,batch", list(zip(DIMS, BATCH)))
def test_forward_layer_by_layer(dims, batch):
    """Every activation, pre-activation and output of the forward pass lies
    in its interval around the exact value computed from the GPU's own
    inputs to that layer."""
    dev = _dev()
    rng = np.random.default_rng(11)
    theta = mlp_ref.init(*dims[:3], seed=5, n_out=dims[3])
    theta[-dims[3]:] = rng.normal(0, 0.2, dims[3])
    xb = _bf16_bits(rng.normal(0, 1, (batch, dims[0])))
    net = _net(dims, batch)
    net.set_params(theta)
    y = net.forward(torch.tensor(xb, device=dev)).cpu().numpy().astype(np.float64)
    layers = _layers(net, theta)
    a = _bits_to_f(xb)
    n_checked = 0
    for l, (W, b) in enumerate(layers):
        s, B = _dot_interval(a, W.T, b)
        if l < len(layers) - 1:
            pre = _bits_to_f(net.intermediate(net.PRE, l, batch))
            act = _bits_to_f(net.intermediate(net.ACT, l, batch))
            ok_pre = _in_bf16_interval(pre, s - B, s + B)
            g = _gelu_exact(s)
            slack = 1.13 * B + 1e-6 * np.abs(s) + 1e-7
            ok_act = _in_bf16_interval(act, g - slack, g + slack)
            print(f"layer {l}: {ok_pre.size} pre-activations, {ok_act.size} activations; "
                  f"outside: {np.count_nonzero(~ok_pre)}, {np.count_nonzero(~ok_act)}")
            assert ok_pre.all() and ok_act.all(), (l, np.argwhere(~ok_pre)[:5], np.argwhere(~ok_act)[:5])
            n_checked += ok_pre.size + ok_act.size
            a = act
        else:
            err = np.abs(y - s)
            print(f"output: max |y - exact| / bound = {np.max(err / B):.3f}")
            assert np.all(err <= B)
            n_checked += y.size
    assert n_checked > 0
    # whole network against the BF16 oracle (flips spread; norm bars)
    ref, (ref_acts, _, _) = mlp_ref.forward(theta, _bits_to_f(xb), dims, bf=True)
    ref_fp64, _ = mlp_ref.forward(theta, _bits_to_f(xb), dims, bf=False)
    e = _rel(y, ref)
    _, Bref = _dot_interval(ref_acts[-1], layers[-1][0].T, layers[-1][1])
    n_out = int(np.count_nonzero(np.abs(y - ref) > Bref))
    print(f"forward dims={dims} batch={batch}: rel L2 vs bf16 oracle {e:.2e}, "
          f"bf16 oracle vs fp64 {_rel(ref, ref_fp64):.2e}; {n_out} of {y.size} outputs "
          f"outside the no-flip interval (BF16 flips upstream)")
    assert e <= 3e-3
    if batch >= 100:
        assert e < 0.2 * _rel(ref, ref_fp64)
    net.close()


def _loss_dz_interval(yg, yt, F, B):
    """Interval of the BF16 loss gradient dz of the output layer (k_loss)
    from the GPU's FP32 outputs yg [B, >= 2F] and the FP32 targets yt."""
    mu, s = yg[:, :F], yg[:, F:2 * F]
    r = yt - mu                                   # exact in FP64
    e = np.exp(-s)
    v_mean = -2.0 * r / B
    d_mean = 4 * U32 * np.abs(v_mean) + 1e-30
    v_var = (1.0 - r * r * e) / B
    d_var = (2e-6 * r * r * e + 4 * U32 * (1.0 + r * r * e)) / B + 1e-30
    lo = np.concatenate([v_mean - d_mean, v_var - d_var], 1)
    hi = np.concatenate([v_mean + d_mean, v_var + d_var], 1)
    return lo, hi


@pytest.mark.parametrize("dims,batch", list(zip(DIMS, BATCH)))
def test_gradients_layer_by_layer(dims, batch):
    """Every backpropagated gradient and every weight and bias gradient lies
    in its interval around the exact value computed from the GPU's own
    stored inputs to that step; the loss and the whole gradient also stay
    close to the BF16 oracle's."""
    dev = _dev()
    rng = np.random.default_rng(12)
    F = dims[3] // 2
    theta = mlp_ref.init(*dims[:3], seed=6, n_out=dims[3])
    theta[-dims[3]:] = rng.normal(0, 0.2, dims[3])
    x = rng.normal(0, 1, (batch, dims[0]))
    yt = rng.normal(0, 1, (batch, F)).astype(np.float32).astype(np.float64)
    xb = _bf16_bits(x)
    net = _net(dims, batch)
    net.set_params(theta)
    xd = torch.tensor(xb, device=dev)
    g, loss = net.gradients(xd, torch.tensor(yt, dtype=torch.float32, device=dev))
    g = g.astype(np.float64)
    layers = _layers(net, theta)
    L = len(layers)
    depth = dims[2]
    # the forward pass of this call: stored activations and pre-activations
    acts = [_bits_to_f(xb)] + [_bits_to_f(net.intermediate(net.ACT, l, batch)) for l in range(depth)]
    pres = [_bits_to_f(net.intermediate(net.PRE, l, batch)) for l in range(depth)]
    yg = np.asarray(net.forward(xd).cpu().numpy(), np.float64)   # same inputs: same outputs
    # output-layer gradient: from the GPU's outputs by the loss definition
    dz_lo, dz_hi = _loss_dz_interval(yg, yt, F, batch)
    dzL = _bits_to_f(net.intermediate(net.DZ, depth, batch))[:, :dims[3]]
    ok = _in_bf16_interval(dzL[:, :F], dz_lo[:, :F], dz_hi[:, :F])
    assert ok.all()
    assert np.all(dzL[:, F:] == 0.0)            # log variances: output layer only
    offs = np.cumsum([0] + [n * k + n for n, k in mlp_ref.shapes(*dims[:3], n_out=dims[3])])
    for l in range(L - 1, -1, -1):
        W, _ = layers[l]
        n_out, k_in = W.shape
        gW = g[offs[l]:offs[l] + n_out * k_in].reshape(n_out, k_in)
        gb = g[offs[l] + n_out * k_in:offs[l + 1]]
        a = acts[l]
        if l == L - 1:
            # the log-variance columns were zeroed after this layer's own
            # gradients: take them as intervals from the loss definition
            lo = np.concatenate([dzL[:, :F], _bf(dz_lo[:, F:])], 1)
            hi = np.concatenate([dzL[:, :F], _bf(dz_hi[:, F:])], 1)
        else:
            lo = hi = _bits_to_f(net.intermediate(net.DZ, l, batch))
        # weight gradient dz^T a: interval sum over the batch + FP32 accumulation
        ap, an = np.maximum(a, 0.0), np.minimum(a, 0.0)
        p_lo = lo.T @ ap + hi.T @ an
        p_hi = hi.T @ ap + lo.T @ an
        mag = (np.maximum(np.abs(lo), np.abs(hi)).T @ np.abs(a))
        Bw = (_gamma(batch + 16) + batch * 2.0 ** -53) * mag + 1e-30
        okW = (gW >= p_lo - Bw) & (gW <= p_hi + Bw)
        Bb = (_gamma(batch + 64) + batch * 2.0 ** -53) * np.maximum(np.abs(lo), np.abs(hi)).sum(0) + 1e-30
        okb = (gb >= lo.sum(0) - Bb) & (gb <= hi.sum(0) + Bb)
        print(f"layer {l}: {gW.size} weight and {gb.size} bias gradients, outside "
              f"{np.count_nonzero(~okW)} / {np.count_nonzero(~okb)}")
        assert okW.all() and okb.all(), (l, np.argwhere(~okW)[:5], np.argwhere(~okb)[:5])
        if l > 0:
            # backpropagated gradient into the previous GELU
            dz = _bits_to_f(net.intermediate(net.DZ, l, batch))[:, :n_out]
            s, Bs = _dot_interval(dz, W)
            z = pres[l - 1]
            gd = mlp_ref.gelu_d(z)
            v = s * gd
            slack = Bs * np.abs(gd) + (np.abs(s) + Bs) * (1e-6 * np.abs(z) + 1e-7) + U32 * np.abs(v)
            got = _bits_to_f(net.intermediate(net.DZ, l - 1, batch))
            okd = _in_bf16_interval(got, v - slack, v + slack)
            print(f"  dz into layer {l - 1}: {okd.size}, outside {np.count_nonzero(~okd)}")
            assert okd.all(), (l, np.argwhere(~okd)[:5])
    # whole network against the BF16 oracle
    rl, rg = mlp_ref.loss_and_grad(theta, _bits_to_f(xb), yt, dims, bf=True)
    _, rg64 = mlp_ref.loss_and_grad(theta, _bits_to_f(xb), yt, dims, bf=False)
    assert abs(loss - rl) <= 1e-3 * max(1.0, abs(rl))
    o = 0
    for n, k in mlp_ref.shapes(*dims[:3], n_out=dims[3]):
        for size in (n * k, n):
            e = _rel(g[o:o + size], rg[o:o + size])
            gap = _rel(rg[o:o + size], rg64[o:o + size])
            print(f"grad block @{o} size {size}: rel L2 {e:.2e} (bf16 vs fp64 {gap:.2e})")
            assert e <= 3e-3, (o, size, e)
            if batch >= 100:
                assert e < 0.3 * gap, (o, size, e, gap)
            o += size
    assert o == g.size
    net.close()


def test_infer_ensemble_matches_member_forwards():
    """dfhm_mlp_infer_ensemble over members the one-launch kernel covers
    (width 512 and 256) and one it does not (width 136): the fluxes equal
    dfhm_mlp_decode_ensemble of the members' dfhm_mlp_forward outputs bit for
    bit, the error estimate is max_f of the member-mean estimate, and
    members with different inputs are refused."""
    dev = _dev()
    rng = np.random.default_rng(19)
    batch = 2999
    nets = []
    for width, seed in ((512, 21), (256, 22), (136, 23)):
        dims = (584, width, 3, 8)
        theta = mlp_ref.init(*dims[:3], seed=seed, n_out=8)
        theta[-8:] = rng.normal(0, 0.2, 8)
        theta[-4:] -= 8.0
        net = _net(dims, batch, seed=seed)
        net.set_params(theta)
        nets.append(net)
    from paper_1703_10119_amd import surrogate
    x = torch.tensor(_bf16_bits(rng.normal(0, 1, (batch, 584))), device=dev)
    scale = np.array([0.1, 1.2, -0.3, 0.9, 1.0, 0.5, -14.0, 0.8], np.float32)
    flux = torch.empty((batch, 2), dtype=torch.float32, device=dev)
    err = torch.empty(batch, dtype=torch.float32, device=dev)
    surrogate.infer_ensemble(nets, x, scale, flux, err)
    ys = [n.forward(x) for n in nets]
    ptrs = (C.c_void_p * 3)(*[y.data_ptr() for y in ys])
    f2 = torch.empty((batch, 2), dtype=torch.float32, device=dev)
    fb = torch.empty(batch, dtype=torch.uint8, device=dev)
    st = dfhm.load().dfhm_mlp_decode_ensemble(ptrs, 3, batch, scale.ctypes.data_as(C.c_void_p), 0.01,
                                              f2.data_ptr(), fb.data_ptr(),
                                              torch.cuda.current_stream().cuda_stream)
    assert st == 0
    torch.cuda.synchronize()
    assert torch.equal(flux, f2)
    m, sd = scale[0::2].astype(np.float64), scale[1::2].astype(np.float64)
    e = np.zeros((batch, 2))
    fks, lgs = [], []
    for y in ys:
        yv = y.cpu().numpy().astype(np.float64)
        u = yv[:, :2] * sd[:2] + m[:2]
        lg = yv[:, 2:4] * sd[2:] + m[2:]
        fks.append(u * np.exp(lg))
        lgs.append(lg)
        e += sd[:2] * np.exp(0.5 * yv[:, 4:6]) + np.abs(u) * sd[2:] * np.exp(0.5 * yv[:, 6:8])
    dis = np.std(np.array(fks), axis=0) / np.exp(np.mean(np.array(lgs), axis=0))
    e = np.sqrt((e / 3) ** 2 + dis ** 2).max(1)
    got = err.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - e) <= 1e-5 * e + 1e-6 * np.abs(m[:2]).max() * sd[2:].max())
    assert np.array_equal(fb.cpu().numpy().astype(bool), ~(got <= 0.01))
    other = _net((40, 256, 2, 8), batch)
    with pytest.raises(dfhm.DfhmError):
        surrogate.infer_ensemble([nets[0], other], x, scale, flux, err)
    for n in nets + [other]:
        n.close()


def test_infer_matches_forward_and_decode():
    """dfhm_mlp_infer = the network's forward pass followed by the flux
    decode: the same fluxes as dfhm_mlp_forward + dfhm_mlp_decode bit for bit,
    and the predicted error max_f sd(u_f) + |u_f| sd(l_f) by its definition
    from the forward outputs."""
    dev = _dev()
    rng = np.random.default_rng(18)
    dims, batch = (584, 512, 4, 8), 3001
    theta = mlp_ref.init(*dims[:3], seed=8, n_out=8)
    theta[-8:] = rng.normal(0, 0.2, 8)
    theta[-4:] -= 8.0                        # log variances around -8
    net = _net(dims, batch)
    net.set_params(theta)
    x = torch.tensor(_bf16_bits(rng.normal(0, 1, (batch, dims[0]))), device=dev)
    scale = np.array([0.1, 1.2, -0.3, 0.9, 1.0, 0.5, -14.0, 0.8], np.float32)
    flux, err = net.infer(x, scale)
    y = net.forward(x)
    f2 = torch.empty((batch, 2), dtype=torch.float32, device=dev)
    fb = torch.empty(batch, dtype=torch.uint8, device=dev)
    st = dfhm.load().dfhm_mlp_decode(y.data_ptr(), batch, scale.ctypes.data_as(C.c_void_p), 0.01,
                                     f2.data_ptr(), fb.data_ptr(),
                                     torch.cuda.current_stream().cuda_stream)
    assert st == 0
    torch.cuda.synchronize()
    assert torch.equal(flux, f2)
    yv = y.cpu().numpy().astype(np.float64)
    m, sd = scale[0::2].astype(np.float64), scale[1::2].astype(np.float64)
    u = yv[:, :2] * sd[:2] + m[:2]
    e = (sd[:2] * np.exp(0.5 * yv[:, 4:6]) + np.abs(u) * sd[2:] * np.exp(0.5 * yv[:, 6:8])).max(1)
    got = err.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - e) <= 1e-5 * e + 1e-6 * np.abs(m[:2]).max() * sd[2:].max())
    assert np.array_equal(fb.cpu().numpy().astype(bool), got > 0.01)
    # argument errors
    bad = scale.copy()
    bad[3] = -1.0
    with pytest.raises(dfhm.DfhmError):
        net.infer(x, bad)
    net.close()
    net4 = _net((40, 136, 2, 4), 16)
    with pytest.raises(dfhm.DfhmError):
        net4.infer(torch.zeros((16, 40), dtype=torch.int16, device=dev), scale)   # n_out != 8
    net4.close()


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
    """Ensemble decode against its definition: the flux is the members' mean,
    the predicted error their mean estimate and their disagreement in
    quadrature; one member gives dfhm_mlp_decode's results bit for bit; bad
    member counts or a null member are refused."""
    dev = _dev()
    rng = np.random.default_rng(17)
    B, K = 777, 3
    ys = []
    base = rng.normal(0, 1, (B, 4))
    for _ in range(K):
        # members that agree to a few 1e-3 (so that their disagreement and
        # their variance heads both matter near tau)
        y = np.empty((B, 8), np.float32)
        y[:, :4] = base + rng.normal(0, 3e-3, (B, 4))
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
    fks, lgs = [], []
    for y in ys:
        yv = y.astype(np.float64)
        u = yv[:, :2] * sd[:2] + m[:2]
        lg = yv[:, 2:4] * sd[2:] + m[2:]
        want += u * np.exp(lg) / K
        fks.append(u * np.exp(lg))
        lgs.append(lg)
        e += (sd[:2] * np.exp(0.5 * yv[:, 4:6]) + np.abs(u) * sd[2:] * np.exp(0.5 * yv[:, 6:8])) / K
        bound += (1e-6 * (np.abs(yv[:, :2] * sd[:2]) + np.abs(m[:2])) * np.exp(lg)
                  + 1e-5 * np.abs(u * np.exp(lg))) / K
    # the members' disagreement over their mean predicted RMS, in quadrature
    dis = np.std(np.array(fks), axis=0) / np.exp(np.mean(np.array(lgs), axis=0))
    e = np.sqrt(e ** 2 + dis ** 2)
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
        c = dfhm.MlpConfig(kw["n_in"], kw["width"], kw["depth"], kw["n_out"], kw["max_batch"],
                           0, 0.9, 0.999, 1e-8, 0.0, None)
        assert L.dfhm_mlp_create(C.byref(c), C.byref(h)) == 1, bad     # DFHM_E_INVAL
    net = S.MLP(n_in=16, width=16, depth=1, n_out=4, max_batch=8)
    x = torch.zeros((9, 16), dtype=torch.int16, device="cuda")
    with pytest.raises(dfhm.DfhmError):
        net.forward(x)                                    # batch above max_batch
    net.close()
