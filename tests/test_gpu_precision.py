"""Precision study on the GPU (the stress configuration and warm-restart drift); the table of
measured errors is printed.  Bounds: an all-FP64 GPU run matches the FP64 oracle to 1e-9 on every
level but the coarsest (layer piston: 1e-7; measured 1.4e-9 and 2.2e-9 on two runs) and on what the
sensors see; FP32 storage with FP64 reductions keeps what the sensors see (A c) within 1e-4, the
residual norms within 1e-5 and every wavelet level but the coarsest within 1e-4 of the oracle
after 12 cold iterations on 35 layers (measured 1.7e-5).  The coarsest level holds layer piston,
fixed by the prior alone, where FP32 rounding is amplified to an O(1) error (measured 0.67, and
0.45-0.49 over all of c): those are held under ceilings of 1.0 and 0.7, so that a change shows up.
The carried FP32 residual stays within 1e-4 of b - M c (relative to ||b||) over 16 warm frames."""
import json

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.timeout(600)  # the oracle's preconditioner probes 770 bands of the stress configuration
def test_stress_precision():
    _need_gpu()
    from tests.precision_study import stress
    r = stress()
    print(json.dumps(r), flush=True)
    # FP64: every level the data constrain, what the sensors see and the residual recurrence to
    # 1e-9; the coarsest level (layer piston, fixed by the prior alone) amplifies rounding by the
    # same factor (~1e7) that turns FP32 rounding into its O(1) error there: 1.1e-16 x 1e7 ~ 1e-9,
    # bounded at 1e-7
    assert max(r["fp64"]["c_by_level"][:-1]) <= 1e-9 and r["fp64"]["visible"]["norm"] <= 1e-9
    assert r["fp64"]["c_by_level"][-1] <= 1e-7
    assert max(r["fp64"]["resnorm_per_iter"]) <= 1e-9
    # FP32: what the sensors see and the residual recurrence follow the oracle; the error sits in
    # the coarsest level (layer piston, constrained by the prior alone) and is reported
    assert r["fp32"]["visible"]["norm"] <= 1e-4
    assert max(r["fp32"]["resnorm_per_iter"]) <= 1e-5
    assert max(r["fp32"]["c_by_level"][:-1]) <= 1e-4
    assert r["fp32"]["c_by_level"][-1] <= 1.0 and r["fp32"]["c"]["norm"] <= 0.7


@pytest.mark.timeout(300)
def test_warm_restart_drift():
    _need_gpu()
    from tests.precision_study import drift
    r = drift(frames=16)
    print(json.dumps(r), flush=True)
    assert max(r["fp64"]["carried_vs_recomputed_residual_over_b"]) <= 1e-10
    assert max(r["fp32"]["carried_vs_recomputed_residual_over_b"]) <= 1e-4


@pytest.mark.timeout(300)
def test_warm_restart_refresh():
    """FEWHA_REFRESH on every 8th frame: the residual recomputed as b - M c brings the carried FP32
    residual back to the level a cold frame leaves (the drift restarts from there)."""
    _need_gpu()
    from tests.precision_study import drift
    r = drift(frames=25, precisions=("fp32",), refresh_every=8)
    print(json.dumps(r), flush=True)
    rows = r["fp32"]["carried_vs_recomputed_residual_over_b"]
    assert max(rows) <= 1e-4
    for f in (8, 16, 24):
        assert rows[f] <= 2 * rows[0], (f, rows[f], rows[0])
