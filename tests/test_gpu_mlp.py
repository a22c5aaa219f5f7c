"""Cost-model kernels against the CPU reference (oracle/mlp.py)."""
import numpy as np
import pytest
import torch

from oracle import mlp
from paper_2508_20403_amd import gss, synth
from tests.gpu_util import assert_same_recovery, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


def test_fp32_gradient_matches_cpu(gpu_ctx):
    rng = np.random.default_rng(0)
    for seed, nb in ((1, 64), (2, 17), (3, 1)):
        w = mlp.random_weights(seed)
        gpu_ctx.costmodel_load(w.astype(np.float32))
        w32 = w.astype(np.float32).astype(np.float64)
        x = rng.normal(0, 2, (nb, mlp.NF)).astype(np.float32)
        y = rng.normal(12, 3, nb).astype(np.float32)
        g_gpu, l_gpu = gpu_ctx.costmodel_grad(x, y)
        l_cpu, g_cpu = mlp.loss_and_grad(w32, x.astype(np.float64), y.astype(np.float64))
        assert abs(l_gpu - l_cpu) <= 1e-4 * max(1.0, abs(l_cpu))
        err = np.abs(g_gpu - g_cpu)
        assert np.linalg.norm(err) <= 1e-4 * np.linalg.norm(g_cpu), (seed, np.linalg.norm(err), np.linalg.norm(g_cpu))
        assert np.all(err <= 1e-4 * np.abs(g_cpu) + 1e-4 * np.abs(g_cpu).max())


def test_bf16_inference_close_to_fp64(gpu_ctx):
    rng = np.random.default_rng(5)
    w = mlp.random_weights(7, scale=0.5)
    gpu_ctx.costmodel_load(w.astype(np.float32))
    for n in (1, 15, 64, 1000, 4097):
        x = rng.normal(0, 1.5, (n, mlp.NF)).astype(np.float32)
        y_cpu, _ = mlp.forward(w.astype(np.float32).astype(np.float64), x.astype(np.float64))
        y_gpu = gpu_ctx.costmodel_predict(torch.from_numpy(x).cuda()).cpu().numpy()
        scale = np.abs(y_cpu).mean() + 1e-3
        assert np.all(np.abs(y_gpu - y_cpu) <= 2e-2 * (np.abs(y_cpu) + scale)), (n, np.abs(y_gpu - y_cpu).max(), scale)


def test_training_fits_a_smooth_target(gpu_ctx):
    rng = np.random.default_rng(11)
    n = 4096
    x = rng.normal(0, 1, (n, mlp.NF)).astype(np.float32)
    logc = 10 + 2 * x[:, 0] + np.abs(x[:, 1]) - 0.5 * x[:, 2] * x[:, 3]
    cyc = np.exp2(logc).astype(np.float64)
    loss = gpu_ctx.costmodel_train(x, cyc, epochs=30, lr=3e-3, seed=1)
    assert np.all(np.isfinite(loss))
    assert loss[-1] < 0.1 * np.var(logc), (loss[0], loss[-1], np.var(logc))
    w = gpu_ctx.costmodel_save()
    y_cpu, _ = mlp.forward(w.astype(np.float64), x.astype(np.float64))
    assert np.mean((y_cpu - logc) ** 2) < 0.15 * np.var(logc)


def test_data_parallel_training_is_deterministic(gpu_ctx):
    """A training set large enough for several 64-sample slices per mini-batch (40000
    rows: two workgroups per step): the fixed-order gradient sum makes two runs with one
    seed give bit-identical weights, and the fit still converges."""
    rng = np.random.default_rng(12)
    n = 40000
    x = rng.normal(0, 1, (n, mlp.NF)).astype(np.float32)
    logc = 10 + 2 * x[:, 0] + np.abs(x[:, 1]) - 0.5 * x[:, 2] * x[:, 3]
    cyc = np.exp2(logc).astype(np.float64)
    loss1 = gpu_ctx.costmodel_train(x, cyc, epochs=8, lr=3e-3, seed=4)
    w1 = gpu_ctx.costmodel_save()
    loss2 = gpu_ctx.costmodel_train(x, cyc, epochs=8, lr=3e-3, seed=4)
    w2 = gpu_ctx.costmodel_save()
    assert np.array_equal(w1.view(np.uint32), w2.view(np.uint32))
    assert np.array_equal(loss1, loss2)
    assert loss1[-1] < 0.5 * loss1[0] and loss1[-1] < 0.1 * np.var(logc), (loss1, np.var(logc))
    y_cpu, _ = mlp.forward(w1.astype(np.float64), x.astype(np.float64))
    assert np.mean((y_cpu - logc) ** 2) < 0.15 * np.var(logc)


def test_learned_schedule_is_bit_exact(gpu_ctx):
    g = synth.config("grid3d_32")
    gpu_ctx.trace_clear()
    gss_tree = gss.Tree.from_graph(gpu_ctx, g)
    gss_tree.recover(g.alpha, g.beta, record=True)
    gss_tree.free()
    feat, cyc, size = gpu_ctx.trace_read()
    gpu_ctx.trace_clear()
    gpu_ctx.costmodel_train(feat, cyc, epochs=5, lr=1e-3, seed=3)
    orc = run_oracle(g)
    for sched in (gss.SCHED_LEARNED, gss.SCHED_EDGECOUNT):
        gpu = run_gpu(gpu_ctx, g, sched=sched)
        assert_same_recovery(gpu, orc)


def test_trained_model_beats_edge_count_on_held_out_subtasks(gpu_ctx):
    """What the trained network gains over the schedule without it: on subtasks it never
    saw (split by feature row, so repeated recordings of one subtask stay on one side),
    its median |log2(predicted / measured cycles)| is below that of the best
    least-squares fit of log2(cycles) on log2(1 + edge count), the only information the
    edge-count schedule has."""
    graphs = synth.batch_config(count=8, nmin=2e4, nmax=2e5, seed=1)
    b = gss.Batch(gpu_ctx, graphs)
    gpu_ctx.set_tuning(256, 1024)
    try:
        gpu_ctx.trace_clear()
        for _ in range(3):
            b.recover(record=True)
        feat, cyc, size = gpu_ctx.trace_read()
        gpu_ctx.trace_clear()
    finally:
        gpu_ctx.set_tuning(64, 2048)
        b.free()
    assert len(cyc) > 1000
    key = np.frombuffer(feat.tobytes(), np.uint32).reshape(len(cyc), -1).astype(np.uint64)
    key = (key * np.uint64(0x9E3779B1)).sum(axis=1) % np.uint64(5)
    held, fit = key == 0, key != 0
    gpu_ctx.costmodel_train(feat[fit], cyc[fit], epochs=20, lr=1e-3, seed=0)
    pred = gpu_ctx.costmodel_predict(torch.from_numpy(np.ascontiguousarray(feat[held])).cuda()).cpu().numpy()
    y = np.log2(np.maximum(cyc, 1.0))
    A = np.stack([np.ones(len(cyc)), np.log2(1.0 + size)], axis=1)
    coef = np.linalg.lstsq(A[fit], y[fit], rcond=None)[0]
    err_mlp = np.median(np.abs(pred - y[held]))
    err_cnt = np.median(np.abs(A[held] @ coef - y[held]))
    print(f"held-out median |log2 error|: network {err_mlp:.3f}, edge-count fit {err_cnt:.3f}")
    assert err_mlp < err_cnt, (err_mlp, err_cnt)


def _adam_reference(w0, x, y, steps, lr):
    """Full-batch Adam in float64 (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected,
    moments from zero) on the float64 mean-squared-error gradient of oracle/mlp.py."""
    P = mlp.NPARAM
    w = np.array(w0, np.float64)
    m = np.zeros(P)
    v = np.zeros(P)
    for t in range(1, steps + 1):
        _, g = mlp.loss_and_grad(w, x, y)
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g * g
        w[:P] -= lr * (m / (1 - 0.9 ** t)) / (np.sqrt(v / (1 - 0.999 ** t)) + 1e-8)
    return w


def test_adam_steps_match_float64(gpu_ctx):
    """Four training steps of the FP32 kernels (one 64-sample mini-batch per epoch, warm
    start from known weights) against four float64 Adam steps.  Tolerance: 2e-3 lr + 1e-6
    |w| per parameter; FP32 gradients and moments move a weight by about 1e-4 lr over four
    steps, while a wrong moment, bias correction or epsilon moves it by a sizeable share
    of lr."""
    rng = np.random.default_rng(21)
    lr = 1e-3
    for seed in (3, 4):
        w0 = mlp.random_weights(seed).astype(np.float32)
        gpu_ctx.costmodel_load(w0)
        x = rng.normal(0, 2, (64, mlp.NF)).astype(np.float32)
        y = np.clip(rng.normal(12, 3, 64), 1, 30).astype(np.float32)
        gpu_ctx.costmodel_train(x, np.exp2(y.astype(np.float64)), epochs=4, lr=lr, seed=seed, warm=True)
        w_gpu = gpu_ctx.costmodel_save().astype(np.float64)
        w_ref = _adam_reference(w0.astype(np.float64), x.astype(np.float64), y.astype(np.float64), 4, lr)
        # the warm start keeps the loaded feature normalisation
        np.testing.assert_array_equal(w_gpu[mlp.NPARAM:], w0[mlp.NPARAM:].astype(np.float64))
        d = np.abs(w_gpu - w_ref)[: mlp.NPARAM]
        assert np.all(d <= 2e-3 * lr + 1e-6 * np.abs(w_ref[: mlp.NPARAM])), (seed, d.max() / lr)
        # and the step moved the weights: about lr per parameter with a gradient
        moved = np.abs(w_ref - w0.astype(np.float64))[: mlp.NPARAM]
        assert np.median(moved) > lr
