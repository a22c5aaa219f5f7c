"""LCA-subtask work queue: the output must not depend on the schedule (queue order,
local/global split, number of workgroups), and the recorder must deliver per-subtask
features and cycles."""
import numpy as np
import pytest

from paper_2508_20403_amd import gss, synth
from tests.gpu_util import assert_same_recovery, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

GRAPHS = [
    lambda: synth.config("grid3d_32"),
    lambda: synth.config("rmat14"),
    lambda: synth.random_connected(3000, 9000, seed=5, alpha=0.2, beta=3, tree="random"),
    lambda: synth.grid((40, 50), 1.0, 1.0, seed=0, alpha=0.2, beta=2, name="unitgrid"),
]


@pytest.mark.parametrize("make", GRAPHS, ids=["grid32", "rmat14", "rand3000", "unitgrid"])
def test_output_independent_of_schedule(gpu_ctx, make):
    g = make()
    orc = run_oracle(g)
    try:
        for local_max, blocks in ((1024, 2048), (0, 2048), (1, 2048), (64, 3), (300, 1), (1024, 7)):
            gpu_ctx.set_tuning(local_max, blocks)
            gpu = run_gpu(gpu_ctx, g)
            assert_same_recovery(gpu, orc)
    finally:
        gpu_ctx.set_tuning(64, 2048)


def test_trace_records_features_and_cycles(gpu_ctx):
    g = synth.config("grid3d_32")
    gpu_ctx.trace_clear()
    tree = gss.Tree.from_graph(gpu_ctx, g)
    st, mask, order, _, info = tree.recover(g.alpha, g.beta, record=True)
    tree.free()
    feat, cyc, size = gpu_ctx.trace_read()
    assert len(cyc) > 0 and np.all(cyc > 0)
    assert np.all(np.isfinite(feat))
    assert np.all(size >= 1) and np.all(size <= 1024)
    # feature 0 is log2(1 + size)
    np.testing.assert_allclose(feat[:, 0], np.log2(1.0 + size), rtol=1e-6)
    gpu_ctx.trace_clear()
    assert len(gpu_ctx.trace_read()[1]) == 0
