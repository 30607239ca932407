"""Launch timing of the step kernels (gmf_set_timing, gmf_get_timing,
gmf_get_timing_by_kind): the window splits into the launches that run
block-step tiles and the update-only launches, the parts add up to the
totals, and gmf_get_timing starts a new window."""
import pytest

from synth import gen_nb

from tests.gpu_helpers import gpu_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_20509_amd import gmf  # noqa: F401  raises if libgmf.so is missing


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_timing_by_kind_splits_the_window(precision):
    pr = gen_nb(n=2000, m=600, d=5, R=4, S=3, seed=1971)
    print(f"[case] timing by kind {precision}", flush=True)
    g = gpu_for(pr, precision=precision)
    g.set_timing(True)
    g.step(2 * 12)
    (tms, tn), (ums, un) = g.get_timing_by_kind()
    ms, n, steps = g.get_timing()
    assert steps == 24
    assert tn >= 1 and un >= 1 and tn + un == n
    assert tms > 0 and ums > 0 and abs(tms + ums - ms) <= 1e-9 * ms + 1e-12
    (tms2, tn2), (ums2, un2) = g.get_timing_by_kind()
    assert tn2 == un2 == 0 and tms2 == ums2 == 0.0
    g.set_timing(False)
    g.close()
