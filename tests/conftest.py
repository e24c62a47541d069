import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def pytest_terminal_summary(terminalreporter):
    """One line over every step-chained parity run of the session: the worst
    step error and how many device decisions fell inside the FP32 band."""
    mod = sys.modules.get("chained")
    reps = [r for _, r in getattr(mod, "REPORTS", [])] if mod else []
    if not reps:
        return
    tot = {k: sum(r[k] for r in reps) for k in ("steps", "hio_band_px", "sw_band_px", "area_band_px",
                                                 "xover_children", "xover_flagged", "selections")}
    terminalreporter.write_sep("-", "step-chained parity against the FP64 oracle")
    terminalreporter.write_line(
        f"{len(reps)} runs, {tot['steps']} steps: max step rel L2 {max(r['max_step_rel'] for r in reps):.2e}, "
        f"max fitness rel {max(r['max_err_rel'] for r in reps):.2e} (bars 1e-5); device decisions inside the "
        f"FP32 band: HIO {tot['hio_band_px']} px, shrink-wrap {tot['sw_band_px']} px, support area "
        f"{tot['area_band_px']} px; crossover children {tot['xover_children']} ({tot['xover_flagged']} near-tie "
        f"flagged), selections {tot['selections']}")


@pytest.fixture(scope="session")
def lib():
    """The loaded HIP library (GPU tests only)."""
    from paper_2409_07413_amd import binding
    return binding.load()
