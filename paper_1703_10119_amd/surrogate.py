"""Surface-flux surrogate: an MLP trained on histories the DF solver produces.

Not part of the paper.  The network predicts the next 10-min mean interior
(side 1) surface fluxes of a wall of the identical-grid batch from the 48 h
outdoor history of its side 0 (T and RH every 10 min), five wall parameters
and the time; the Dufort-Frankel solve is both the source of the training
targets and the fallback when the network's own error estimate is too large.
Every kernel (DF steps, feature rows, GEMMs, loss, AdamW, decode) runs on the
GPU through the C ABI; this module only orchestrates calls and computes the
summary statistics.
"""
from __future__ import annotations

import ctypes as C
import json
import math
import time

import numpy as np

from . import dfhm, workloads as wl

N_HIST = 288          # 48 h at 10-min spacing
STRIDE = 584          # feature row: 576 history values + 8 parameters
WINDOW_S = 600.0      # prediction interval
SPINUP_S = 48 * 3600.0
N_WINDOWS = 156       # 26 h of windows after the spin-up


MlpConfig, FeatureDesc = dfhm.MlpConfig, dfhm.FeatureDesc


def _lib():
    return dfhm.load()


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


class MLP:
    """The network on the current device (BF16 MFMA, FP32 master weights)."""

    def __init__(self, n_in=STRIDE, width=512, depth=4, n_out=8, max_batch=65536, seed=0,
                 beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
        L = _lib()
        c = MlpConfig(n_in, width, depth, n_out, max_batch, seed, beta1, beta2, eps,
                      weight_decay, _stream())
        h = C.c_void_p()
        st = L.dfhm_mlp_create(C.byref(c), C.byref(h))
        if st != 0:
            raise dfhm.DfhmError(st, "dfhm_mlp_create")
        self._h = h
        self.dims = (n_in, width, depth, n_out)
        self.n_params = int(L.dfhm_mlp_param_count(h))
        self.max_batch = max_batch

    def _check(self, st, what):
        if st != 0:
            raise dfhm.DfhmError(st, f"{what}: {_lib().dfhm_mlp_last_error(self._h).decode()}")

    def close(self):
        if getattr(self, "_h", None):
            _lib().dfhm_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def forward(self, x):
        import torch
        B = x.shape[0]
        y = torch.empty((B, self.dims[3]), dtype=torch.float32, device=x.device)
        self._check(_lib().dfhm_mlp_forward(self._h, x.data_ptr(), B, y.data_ptr()), "forward")
        return y

    def infer(self, x, scale, noalloc=False):
        """Fluxes [B, 2] and predicted relative errors [B] of the flux head
        (dfhm_mlp_infer, or dfhm_mlp_infer_noalloc); scale = 8 floats."""
        import torch
        B = x.shape[0]
        flux = torch.empty((B, 2), dtype=torch.float32, device=x.device)
        err = torch.empty(B, dtype=torch.float32, device=x.device)
        sc = np.ascontiguousarray(scale, np.float32)
        fn = _lib().dfhm_mlp_infer_noalloc if noalloc else _lib().dfhm_mlp_infer
        self._check(fn(self._h, x.data_ptr(), B, sc.ctypes.data_as(C.c_void_p), flux.data_ptr(),
                       err.data_ptr()), "infer")
        return flux, err

    def noalloc_max_batch(self) -> int:
        return int(_lib().dfhm_mlp_noalloc_max_batch(self._h))

    ACT, PRE, DZ = 0, 1, 2

    def intermediate(self, kind, layer, rows):
        """BF16 bit patterns (uint16 [rows, cols]) of a stored intermediate of
        the last pass (dfhm_mlp_get_intermediate)."""
        n_in, width, depth, n_out = self.dims
        cols = 32 if (kind == self.DZ and layer == depth) else width
        out = np.empty((rows, cols), np.uint16)
        self._check(_lib().dfhm_mlp_get_intermediate(self._h, int(kind), int(layer), int(rows),
                                                     out.ctypes.data_as(C.c_void_p)),
                    "get_intermediate")
        return out

    def train_step(self, x, y, lr, want_loss=False):
        loss = C.c_float(0.0)
        self._check(_lib().dfhm_mlp_train_step(self._h, x.data_ptr(), y.data_ptr(), x.shape[0],
                                               float(lr), C.byref(loss) if want_loss else None),
                    "train_step")
        return float(loss.value) if want_loss else None

    def gradients(self, x, y):
        g = np.empty(self.n_params, np.float32)
        loss = C.c_float(0.0)
        self._check(_lib().dfhm_mlp_gradients(self._h, x.data_ptr(), y.data_ptr(), x.shape[0],
                                              g.ctypes.data_as(C.c_void_p), C.byref(loss)),
                    "gradients")
        return g, float(loss.value)

    def get_params(self):
        p = np.empty(self.n_params, np.float32)
        self._check(_lib().dfhm_mlp_get_params(self._h, p.ctypes.data_as(C.c_void_p)), "get")
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, np.float32)
        self._check(_lib().dfhm_mlp_set_params(self._h, p.ctypes.data_as(C.c_void_p)), "set")


def wall_inputs(walls):
    """Per-wall sinusoids of side 0 [W, 8] and 5 parameters [W, 5]: log10 of
    the four law scales of layer 0 and the wall thickness."""
    W = len(walls["nx"])
    sines = np.concatenate([walls["Tamb"][:, 0, :], walls["RHamb"][:, 0, :]], axis=1)
    F = wl.LAYER_FIELDS
    lay = walls["layer"][:, 0, :]
    params = np.stack([np.log10(lay[:, F.index("k0")]), np.log10(lay[:, F.index("kM0")]),
                       np.log10(lay[:, F.index("c0")]), np.log10(lay[:, F.index("cM0")]),
                       walls["layer"][:, :, F.index("thick")].sum(axis=1)], axis=1)
    return np.ascontiguousarray(sines, np.float64).reshape(W, 8), params.astype(np.float32)


def feature_desc(params, t_lo, t_hi):
    """Normalisation of the feature rows (history around 293 K / RH 0.6;
    parameter means and spreads of the training walls; time over its range)."""
    d = FeatureDesc()
    d.n_hist, d.stride, d.dt_hist = N_HIST, STRIDE, WINDOW_S
    d.T_mean, d.T_scale, d.RH_mean, d.RH_scale = 293.0, 10.0, 0.6, 0.2
    mu = params.mean(axis=0)
    sd = params.std(axis=0)
    for i in range(5):
        d.p_mean[i] = float(mu[i])
        d.p_scale[i] = float(sd[i]) if sd[i] > 1e-6 else 1.0
    d.p_mean[5] = 0.5 * (t_lo + t_hi) / 86400.0
    d.p_scale[5] = max(0.5 * (t_hi - t_lo) / 86400.0, 1e-3)
    for i in (6, 7):
        d.p_mean[i], d.p_scale[i] = 0.0, 0.7071
    return d


def features(wall_idx, t, sines_d, params_d, desc):
    """BF16 feature rows (as int16 torch tensor) of samples (wall, time)."""
    import torch
    n = int(wall_idx.shape[0])
    x = torch.empty((n, STRIDE), dtype=torch.int16, device=wall_idx.device)
    st = _lib().dfhm_mlp_features(wall_idx.data_ptr(), t.data_ptr(), sines_d.data_ptr(),
                                  params_d.data_ptr(), n, C.byref(desc), x.data_ptr(), _stream())
    if st != 0:
        raise dfhm.DfhmError(st, "dfhm_mlp_features")
    return x


def generate(walls, precision=dfhm.FP64, dt=1.0, spinup_s=SPINUP_S, n_windows=N_WINDOWS):
    """Run the DF solver on a wall batch and return the window targets.

    Returns dict(flux [W, n_windows, 2] side-1 mean (heat W/m2, vapour
    kg/(m2 s)), t [n_windows] window start times, df_seconds, steps)."""
    import torch
    cfg = wl.default_config(dt=dt)
    s = dfhm.Solver(walls, cfg, precision=precision, schedule=dfhm.SCHED_RESIDENT)
    spin = int(round(spinup_s / dt))
    wsteps = int(round(WINDOW_S / dt))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(spin)
    _, I_prev = s.fluxes()
    out = np.empty((len(walls["nx"]), n_windows, 2))
    for k in range(n_windows):
        s.step(wsteps)
        _, I = s.fluxes()
        out[:, k, :] = (I[:, 1, :] - I_prev[:, 1, :]) / (wsteps * dt)
        I_prev = I
    s.sync()
    secs = time.perf_counter() - t0
    s.close()
    t_win = spinup_s + WINDOW_S * np.arange(n_windows)
    steps = spin + n_windows * wsteps
    return dict(flux=out, t=t_win, df_seconds=secs, steps=steps,
                cell_updates=float(wl.total_nodes(walls)) * steps, window_steps=wsteps)


class Targets:
    """Per-wall scale split of the window fluxes: u = flux / RMS_w and
    l = log RMS_w per field (RMS over the windows of the wall), each z-scored
    with the training set's mean and std."""

    def __init__(self, flux):
        u, l = self.split(flux)
        self.mean = np.array([u[..., 0].mean(), u[..., 1].mean(), l[..., 0].mean(), l[..., 1].mean()])
        self.std = np.array([u[..., 0].std(), u[..., 1].std(), l[..., 0].std(), l[..., 1].std()])
        self.std = np.where(self.std > 0, self.std, 1.0)

    @staticmethod
    def split(flux):
        rms = np.sqrt(np.mean(flux ** 2, axis=1, keepdims=True))
        rms = np.maximum(rms, 1e-300)
        return flux / rms, np.broadcast_to(np.log(rms), flux.shape)

    def norm(self, flux):
        """[W, K, 2] fluxes -> [W, K, 4] normalised targets (u_q, u_g, l_q, l_g)."""
        u, l = self.split(flux)
        t = np.concatenate([u, l], axis=2)
        return (t - self.mean) / self.std

    def scale8(self):
        return np.array([v for i in range(4) for v in (self.mean[i], self.std[i])], np.float32)


def train(net, data, walls, desc, targets, epochs=3, batch=8192, lr=1e-3, seed=0, log=None):
    """AdamW on all (wall, window) samples of `data`; linear warm-up, then a
    cosine learning-rate decay."""
    import torch
    dev = "cuda"
    sines, params = wall_inputs(walls)
    sines_d = torch.tensor(sines, device=dev)
    params_d = torch.tensor(params, device=dev)
    W, K = data["flux"].shape[:2]
    y_all = torch.tensor(targets.norm(data["flux"]).reshape(-1, 4), dtype=torch.float32, device=dev)
    wall_of = torch.arange(W, device=dev, dtype=torch.int32).repeat_interleave(K)
    t_of = torch.tensor(np.tile(data["t"], W), dtype=torch.float64, device=dev)
    n = W * K
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    steps = epochs * (n // batch)
    warm = max(1, steps // 20)              # linear warm-up over the first 5 %
    k = 0
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g, device=dev)
        for b in range(n // batch):
            idx = perm[b * batch:(b + 1) * batch]
            x = features(wall_of[idx].contiguous(), t_of[idx].contiguous(), sines_d, params_d, desc)
            y = y_all[idx].contiguous()
            cur = lr * min(1.0, (k + 1) / warm) * 0.5 * (1.0 + math.cos(math.pi * k / max(steps, 1)))
            want = (k % 200 == 0) or (k == steps - 1)
            loss = net.train_step(x, y, cur, want_loss=want)
            if want:
                losses.append((k, loss))
                if log and (k % 2000 == 0 or k == steps - 1):
                    log(f"  step {k}/{steps} loss {loss:.4f}")
            k += 1
    torch.cuda.synchronize()
    return dict(losses=losses, seconds=time.perf_counter() - t0, steps=steps, samples=steps * batch)


def infer_ensemble(nets, x, scale, flux, err):
    """Fluxes flux[B, 2] and error estimates err[B] of an ensemble of flux
    heads on features x (dfhm_mlp_infer_ensemble); flux and err are
    preallocated device tensors (views of larger ones allowed)."""
    hs = (C.c_void_p * len(nets))(*[n._h for n in nets])
    sc = np.ascontiguousarray(scale, np.float32)
    st = _lib().dfhm_mlp_infer_ensemble(hs, len(nets), x.data_ptr(), x.shape[0],
                                         sc.ctypes.data_as(C.c_void_p), flux.data_ptr(),
                                         err.data_ptr())
    if st != 0:
        raise dfhm.DfhmError(st, "dfhm_mlp_infer_ensemble: " +
                             _lib().dfhm_mlp_last_error(nets[0]._h).decode())


def predict(nets, walls, t_windows, desc, targets, tau, batch=65536):
    """Network fluxes [W, K, 2] and fallback flags [W, K] for all windows,
    from one network or the mean of an ensemble (a list of networks)."""
    import torch
    nets = list(nets) if isinstance(nets, (list, tuple)) else [nets]
    dev = "cuda"
    sines, params = wall_inputs(walls)
    sines_d = torch.tensor(sines, device=dev)
    params_d = torch.tensor(params, device=dev)
    W, K = len(walls["nx"]), len(t_windows)
    wall_of = torch.arange(W, device=dev, dtype=torch.int32).repeat_interleave(K)
    t_of = torch.tensor(np.tile(t_windows, W), dtype=torch.float64, device=dev)
    n = W * K
    flux = torch.empty((n, 2), dtype=torch.float32, device=dev)
    err = torch.empty(n, dtype=torch.float32, device=dev)
    sc = targets.scale8()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b0 in range(0, n, batch):
        b1 = min(n, b0 + batch)
        x = features(wall_of[b0:b1].contiguous(), t_of[b0:b1].contiguous(), sines_d, params_d, desc)
        infer_ensemble(nets, x, sc, flux[b0:b1], err[b0:b1])
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    fb = ~(err <= float(tau))            # a NaN estimate falls back
    return (flux.cpu().numpy().reshape(W, K, 2).astype(np.float64),
            fb.cpu().numpy().reshape(W, K).astype(bool), secs)


def errors(pred, truth):
    """|pred - truth| / RMS over the windows of the truth, per wall and field."""
    rms = np.sqrt(np.mean(truth ** 2, axis=1, keepdims=True))
    return np.abs(pred - truth) / rms


def calibrate_tau(nets, walls, data, desc, targets, target=0.01, q=0.99):
    """Largest fallback threshold (predicted relative error) whose p-q error
    after fallback is <= target on the given (calibration) walls; a fallback
    sample takes the DF value of `data`, which the fallback solve reproduces
    (checked where the pipeline runs, in `serve`)."""
    for tau in np.geomspace(0.1, 0.0005, 40):
        pred, fb, _ = predict(nets, walls, data["t"], desc, targets, tau)
        e = errors(pred, data["flux"]).max(axis=2)
        e[fb] = 0.0
        if np.quantile(e, q) <= target:
            return float(tau)
    return None


def _timed(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def serve(nets, walls, truth, desc, targets, tau, windows, dt=1.0, precision=dfhm.FP64):
    """The surrogate as a solver, executed and timed against the DF solve.

    A query asks for the next-window mean interior fluxes of every wall at
    window k.  The DF solve answers it by running all walls from their
    initial state to the end of window k (timed once, in one run with
    checkpoints at the query windows).  The surrogate pipeline answers it
    with the networks (feature rows, forward passes, ensemble decode with
    its error estimate), then runs the DF solver from the initial state to
    the end of window k on just the walls whose estimate exceeds tau, and
    takes their DF fluxes.  Both times include creating the solver and
    reading the fluxes back.  Every answer is judged against `truth` (the
    continuous DF run): |answer - truth| / RMS over the windows of the
    truth, per wall and field; the fallback answers are compared too."""
    import torch
    W = len(walls["nx"])
    cfg = wl.default_config(dt=dt)
    wsteps = int(round(WINDOW_S / dt))
    spin = int(round(SPINUP_S / dt))
    windows = sorted(int(k) for k in windows)

    def df_to(sub, ks):
        """DF on wall set `sub` to the end of each window in ks; returns the
        window fluxes [len(sub), len(ks), 2] and the elapsed time at each
        window's end (from before the solver is created)."""
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = dfhm.Solver(sub, cfg, precision=precision, schedule=dfhm.SCHED_RESIDENT)
        n = 0
        out = np.empty((len(sub["nx"]), len(ks), 2))
        at = []
        for i, k in enumerate(ks):
            start = spin + k * wsteps
            s.step(start - n)
            _, I0 = s.fluxes()
            s.step(wsteps)
            _, I1 = s.fluxes()
            n = start + wsteps
            out[:, i, :] = (I1[:, 1, :] - I0[:, 1, :]) / (wsteps * dt)
            at.append(time.perf_counter() - t0)
        s.close()
        return out, at

    base, t_base = df_to(walls, windows)
    rms = np.sqrt(np.mean(truth["flux"] ** 2, axis=1))                 # [W, 2]
    sines, params = wall_inputs(walls)
    dev = "cuda"
    sines_d = torch.tensor(sines, device=dev)
    params_d = torch.tensor(params, device=dev)
    wall_of = torch.arange(W, device=dev, dtype=torch.int32)
    sc = np.ascontiguousarray(targets.scale8())
    rows = []
    for i, k in enumerate(windows):
        t_k = torch.full((W,), SPINUP_S + WINDOW_S * k, dtype=torch.float64, device=dev)

        def network():
            x = features(wall_of, t_k, sines_d, params_d, desc)
            flux = torch.empty((W, 2), dtype=torch.float32, device=dev)
            err = torch.empty(W, dtype=torch.float32, device=dev)
            infer_ensemble(nets, x, sc, flux, err)
            fb = ~(err <= float(tau))        # a NaN estimate falls back
            return flux.cpu().numpy().astype(np.float64), fb.cpu().numpy().astype(bool)

        network()                                   # warm-up (first launch of the kernels)
        (flux, fb), t_net = _timed(network)
        idx = np.nonzero(fb)[0]
        t_fb = 0.0
        if len(idx):
            fl, at = df_to(wl.subset(walls, idx), [k])
            t_fb = at[0]
            fb_err = np.abs(fl[:, 0, :] - truth["flux"][idx, k, :]) / rms[idx]
            flux[idx] = fl[:, 0, :]
        else:
            fb_err = np.zeros((0, 2))
        e = (np.abs(flux - truth["flux"][:, k, :]) / rms).max(axis=1)
        base_err = np.abs(base[:, i, :] - truth["flux"][:, k, :]) / rms
        rows.append(dict(window=k, t_df=t_base[i], t_net=t_net, t_fallback=t_fb,
                         speedup=t_base[i] / (t_net + t_fb), fallback_fraction=len(idx) / W,
                         err_p50=float(np.median(e)), err_p99=float(np.quantile(e, 0.99)),
                         err_max=float(e.max()), fallback_err_max=float(fb_err.max()) if len(idx) else 0.0,
                         df_rerun_err_max=float(base_err.max()),
                         speedup_network_only=t_base[i] / t_net))
    tot_df = sum(r["t_df"] for r in rows)
    tot_sur = sum(r["t_net"] + r["t_fallback"] for r in rows)
    return dict(windows=rows, speedup=tot_df / tot_sur,
                speedup_network_only=tot_df / sum(r["t_net"] for r in rows),
                fallback_fraction=float(np.mean([r["fallback_fraction"] for r in rows])),
                err_p99=max(r["err_p99"] for r in rows), err_max=max(r["err_max"] for r in rows),
                fallback_err_max=max(r["fallback_err_max"] for r in rows),
                df_seconds=tot_df, surrogate_seconds=tot_sur, walls=W)


def study(n_train=65536, n_cal=2048, n_test=8192, epochs=60, lr=2e-3, batch=16384,
          target=0.01, q=0.99, cal_margin=0.9, seed=1, n_nets=3,
          windows=(0, 52, 104, 155), log=None):
    """Train on DF histories, calibrate the fallback threshold on one set of
    walls, and run the executed pipeline (`serve`) on another (all C2-type
    walls: 30 cm, 1001 nodes, dt = 1 s, different generator seeds; FP64 DF
    targets and fallback).  With n_nets > 1 an ensemble of networks (seeds
    seed, seed + 1, ...) is trained on the same data and its mean flux and
    mean predicted error are used; the network time covers every member.

    Error: |q - q_DF| / RMS over the windows of q_DF, per wall and field; a
    sample's error is the larger of its two fields.  tau is the largest
    threshold whose q-quantile error on the calibration walls is <=
    cal_margin * target.  The raw errors (no fallback) are reported over all
    windows of the held-out walls, and the FP32 DF solve's own error against
    the FP64 targets on the calibration walls."""
    say = log or (lambda *a: None)
    tr = wl.uniform_batch(n_train, seed=505)
    ca = wl.uniform_batch(n_cal, seed=515)
    te = wl.uniform_batch(n_test, seed=516)
    d_tr = generate(tr)
    say(f"DF data (FP64): {n_train} walls x {d_tr['steps']} steps in {d_tr['df_seconds']:.1f} s")
    d_ca = generate(ca)
    d_ca32 = generate(ca, precision=dfhm.FP32)
    e32 = errors(d_ca32["flux"], d_ca["flux"])
    d_te = generate(te)
    targets = Targets(d_tr["flux"])
    _, params = wall_inputs(tr)
    desc = feature_desc(params, d_tr["t"][0], d_tr["t"][-1])
    nets = [MLP(max_batch=65536, seed=seed + k) for k in range(n_nets)]
    fits = []
    for k, net in enumerate(nets):
        say(f"training network {k + 1} of {n_nets}")
        fits.append(train(net, d_tr, tr, desc, targets, epochs=epochs, batch=batch, lr=lr,
                          seed=seed + k, log=log))
    fit = dict(steps=sum(f["steps"] for f in fits), seconds=sum(f["seconds"] for f in fits),
               samples=sum(f["samples"] for f in fits))
    n_params = nets[0].n_params
    say(f"trained {fit['steps']} steps of {batch} in {fit['seconds']:.1f} s")
    say("calibrating the fallback threshold")
    tau = calibrate_tau(nets, ca, d_ca, desc, targets, target=cal_margin * target, q=q)
    predict(nets, te, d_te["t"], desc, targets, 10.0)           # warm-up
    pred, _, mlp_s = predict(nets, te, d_te["t"], desc, targets, 10.0)
    e_raw = errors(pred, d_te["flux"]).max(axis=2)
    say(f"serving {len(windows)} query windows of {n_test} walls (tau {tau})")
    sv = serve(nets, te, d_te, desc, targets, tau if tau else 1e-30, windows)
    flops = 2.0 * n_params * e_raw.size * n_nets     # multiply-adds of the forward passes
    for net in nets:
        net.close()
    return dict(
        tau=tau, fallback_fraction=sv["fallback_fraction"], speedup=sv["speedup"],
        speedup_network_only=sv["speedup_network_only"], err_p99=sv["err_p99"],
        err_max=sv["err_max"], fallback_err_max=sv["fallback_err_max"],
        serve_windows=sv["windows"], df_seconds=sv["df_seconds"],
        surrogate_seconds=sv["surrogate_seconds"],
        raw_err_p50=float(np.median(e_raw)), raw_err_p99=float(np.quantile(e_raw, q)),
        raw_frac_above_target=float(np.mean(e_raw > target)),
        fp32_df_err_p99=[float(np.quantile(e32[..., f], 0.99)) for f in range(2)],
        fp32_df_err_max=[float(e32[..., f].max()) for f in range(2)],
        mlp_seconds=mlp_s, mlp_tflops=flops / mlp_s / 1e12, samples=int(e_raw.size),
        train_seconds=fit["seconds"], train_samples=fit["samples"],
        train_tflops=3.0 * 2.0 * n_params * fit["samples"] / fit["seconds"] / 1e12,
        data_seconds=d_tr["df_seconds"], n_train=n_train, n_cal=n_cal, n_test=n_test,
        epochs=epochs, batch=batch, lr=lr, n_nets=n_nets)


def kernel_bench(batch=65536, train_batch=16384, iters=50, seed=0):
    """Time the network's kernels alone on synthetic BF16 inputs: forward at
    the inference batch and one AdamW training step, with HIP events on the
    stream the kernels are launched on.  FLOPs are the GEMMs' multiply-adds
    (2 per weight per sample; x3 for a training step)."""
    import torch
    dev = "cuda"
    net = MLP(max_batch=max(batch, train_batch), seed=seed)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    x = (torch.randn((batch, STRIDE), generator=g, device=dev)
         .to(torch.bfloat16).view(torch.int16).contiguous())
    xt = x[:train_batch].contiguous()
    yt = torch.randn((train_batch, 4), generator=g, device=dev)
    stream = torch.cuda.current_stream()
    n_w = net.n_params - sum(net.dims[1] for _ in range(net.dims[2])) - net.dims[3]
    fwd_flops = 2.0 * n_w

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(n):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3 / n

    scale = np.array([0.0, 1.0, 0.0, 1.0, 0.0, 1.0, 0.0, 1.0], np.float32)
    t_inf = timed(lambda: net.infer(x, scale), iters)
    t_fwd = timed(lambda: net.forward(x), iters)
    t_train = timed(lambda: net.train_step(xt, yt, 1e-4), iters)
    net.close()
    return dict(infer_s=t_inf, infer_tflops=fwd_flops * batch / t_inf / 1e12,
                forward_s=t_fwd, forward_tflops=fwd_flops * batch / t_fwd / 1e12,
                train_step_s=t_train,
                train_tflops=3.0 * fwd_flops * train_batch / t_train / 1e12,
                batch=batch, train_batch=train_batch, flops_per_sample=fwd_flops)


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="surrogate kernel timing")
    ap.add_argument("--iters", type=int, default=50)
    a = ap.parse_args()
    print(json.dumps(kernel_bench(iters=a.iters)), flush=True)
