"""Run metrics from the device counters against the oracle: particle count,
arrivals of the last step (particles whose element changed), smallest and
largest particle count of a cell, error word, steps done."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1003_4548_amd as P
    P.load_library()
    return P


def test_metrics_match_the_oracle(gpu):
    wl = W.tiny_canyon(precision="f32", nens=3)
    print(f"[case] metrics {wl.name} n={wl.n_total}", flush=True)
    sim = gpu.Simulation.from_workload(wl)
    orc = O.Oracle(wl)
    sim.step(4)
    orc.step(4)
    before = [orc.state(en)["elem"] for en in range(wl.nens)]
    sim.step(1)
    orc.step(1)
    m = sim.metrics()
    after = [orc.state(en)["elem"] for en in range(wl.nens)]
    counts = np.concatenate([np.bincount(e, minlength=wl.mesh.nelem) for e in after])
    assert m["particles"] == wl.n_total
    assert m["arrivals_last_step"] == sum(int((a != b).sum()) for a, b in zip(after, before))
    assert m["arrivals_last_step"] > 0
    assert m["min_per_cell"] == counts.min() and m["max_per_cell"] == counts.max()
    assert m["error_word"] == 0 and m["steps_done"] == 5 and m["repacks"] == 0
    assert m["cells_over_three_quarters"] >= 0
