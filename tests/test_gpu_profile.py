"""Per-phase profiling through the C-ABI (sibfa_set_profiling,
sibfa_set_profiling_phases, sibfa_get_profile).

Checks: recording events changes no result (energies and forces
bit-identical with profiling on and off); the real-space matvec phase counts
one launch per product of the context's own precision, and in mixed
precision the FP64 products of the residual replacements are counted under
their own phase (none in FP64); a phase mask times only the named phases;
the list sizes match the neighbour counts."""
import numpy as np
import pytest
import torch

from synth import config_system
from tests.gpu_util import say, gpu_params, engine_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _evaluate(eng, pos):
    eng.update_positions(pos)
    _, it, _ = eng.solve(warm_start=False)
    e_pol, e_elec, f = eng.energy_forces()
    return it, e_pol, e_elec, f.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_profile_phases(precision):
    say(f"[profile] box1024 {precision}")
    d, prm = config_system("box1024")
    eng = engine_for(d, gpu_params(d, beta=prm["beta"], cutoff=prm["cutoff"], grid=prm["grid"],
                                   tol=prm["tol"], precision=precision, precond="molblock"))
    pos = torch.as_tensor(d["pos"], dtype=torch.float64, device="cuda").contiguous()
    ref = _evaluate(eng, pos)

    eng.set_profiling(True)
    got = _evaluate(eng, pos)
    prof = eng.profile()
    eng.set_profiling(False)
    assert got[0] == ref[0]
    assert got[1] == ref[1] and got[2] == ref[2]
    assert np.array_equal(got[3], ref[3])

    ms, calls = prof["ms"], prof["calls"]
    assert all(v >= 0.0 for v in ms.values())
    for name in ("lists", "field_real", "field_recip", "matvec", "update", "force_real",
                 "force_recip", "paircoef", "matvec_recip"):
        assert calls[name] > 0, name
    fp64_products = calls["matvec_fp64"]
    if precision == "mixed":
        # the early replacement and the final check
        assert fp64_products >= 2 and ms["matvec_fp64"] > 0.0
    else:
        assert fp64_products == 0 and ms["matvec_fp64"] == 0.0
    # one real-space launch per product of the context's precision: the
    # iterations plus the residual from scratch (FP64 contexts also count
    # the final check there)
    assert got[0] + 1 <= calls["matvec"] <= got[0] + 3
    counts = eng.neighbor_counts().cpu().numpy()
    assert prof["pairs"]["all"] == int(counts.sum())

    eng.set_profiling(True, phases=["matvec"])
    _evaluate(eng, pos)
    prof = eng.profile()
    eng.set_profiling(False)
    assert prof["calls"]["matvec"] == calls["matvec"]
    assert all(c == 0 for k, c in prof["calls"].items() if k != "matvec")
    eng.close()
