"""What the trained surrogate gains over the DF solve without it (GPU).

A reduced version of the full study (16,384 training walls instead of
65,536): train the networks (an ensemble of three) on DF histories with the
project's kernels, calibrate the fallback threshold on one set of walls,
then on a third set
check that the error after fallback meets the 1 % target at the 99th
percentile and that the surrogate with its DF fallback is faster than the
DF solve alone, with the DF state carried between windows (warm) and
rebuilt for each prediction (cold).  The network and its error target are
not part of the paper (parity unpinned by the paper); the DF solve it is
judged against is the parity-tested GPU path.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_surrogate_gain_at_one_percent_error():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1703_10119_amd import surrogate as S
    r = S.study(n_train=16384, n_cal=1024, n_test=1024, epochs=40, lr=2e-3, batch=8192,
                log=lambda *a: print(*a, flush=True))
    print({k: (round(v, 5) if isinstance(v, float) else v) for k, v in r.items()})
    # the network learned the fluxes: median error well below the raw scale
    assert r["raw_err_p50"] < 0.03
    assert r["tau"] is not None
    # the target is met on walls the threshold was not calibrated on
    assert r["err_p99"] <= 0.01
    # and the surrogate plus fallback beats the solver alone
    assert r["speedup_warm"] > 1.0
    assert r["speedup_cold"] > 1.0
    assert r["speedup_no_fallback_warm"] > 50.0
