"""The per-step timestamp summary (paper_2106_09382_amd.steptimes) on a small
solve: the timed solve takes the same sweeps as the untimed one, and the
summary's step times are positive and ordered."""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2106_09382_amd import _lib
    _lib.load()
    return _lib


def test_step_times_summary(lib):
    from paper_2106_09382_amd import datagen, steptimes
    pr = datagen.problem(2, p=300, n=200)
    Y = torch.from_numpy(pr["y"]).cuda()
    r = steptimes.step_times(Y, 0.2, tol=1e-7, w_in_lds=2, row_groups=16, col_slices=2)
    _, info = lib.fit(Y, 0.2, 1e-7, 500, kind="Y", w_in_lds=2, row_groups=16, col_slices=2)
    assert r["sweeps"] == info["sweeps"] and r["launch"][:2] == [16, 2]
    pc = r["step_us_percentiles"]
    assert 0 < pc["10"] <= pc["50"] <= pc["90"] <= pc["99"]
    assert 0 < r["row_phase_us_mean"] < 10 * r["step_us_mean"]
    assert r["start_spread_us_median"] >= 0
