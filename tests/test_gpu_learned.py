"""What the learned initial guess gains over the method without it.

A U-Net is trained on the GPU (libmcd's BF16-MFMA kernels) on PPE solves of
four seeded cylinder trajectories (128^2 mesh), then every PPE of a held-out
trajectory is solved to the same tolerance from zero, from the previous
pressure (warm start) and from the learned guess, and from zero and the warm
start with the Jacobi preconditioner (the classical comparator).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_17542_amd import learned, mcd
    mcd.load()
    return learned


def test_learned_guess_gain_on_held_out_trajectory(L):
    from paper_2404_17542_amd import configs, mcd as M
    n, ch = 128, (16, 32, 64, 128)
    bc = configs.c2_oscillating_cylinder(n=n).bc_pressure
    data = L.collect(range(1000, 1004), n, n_spin=10, n_save=40, log=lambda *_: None)
    held = L.collect([2000], n, n_spin=10, n_save=8, log=lambda *_: None)
    ctx = M.Context.from_case(configs.c2_oscillating_cylinder(n=n))
    model = M.Model(ctx, ch)
    model.set_params(L.init_theta(ch, 0))
    model.set_output_scale(L.output_scale(data, bc))
    before = L.eval_loss(model, held, bc)
    L.train(model, data, bc, epochs=8, lr=5e-4, seed=0, log=lambda *_: None)
    after = L.eval_loss(model, held, bc)
    # loss 1 is the warm start itself (relative squared error of the correction)
    assert before == pytest.approx(1.0)
    assert after < 0.7, after
    modes = ("zero", "zero+jacobi", "warm+jacobi", "learned", "warm")
    res = L.evaluate(model, [2000], n, n_spin=10, n_eval=8, modes=modes, log=lambda *_: None)
    s = L.summarize(res)
    msg = str(s)
    print(msg)
    # every solve reaches the tolerance whatever the guess
    assert all(np.isfinite(v) for m in modes for v in res[m]["iters"]), msg
    # the network's guess has a smaller initial residual than the warm start ...
    assert s["learned"]["mean_rel0"] < 0.6 * s["warm"]["mean_rel0"], msg
    # ... and needs fewer Bi-CGSTAB iterations than the zero start; against
    # the warm start the iteration count is about the same (measured: within
    # a few per cent either way), which this test records but does not claim
    assert s["learned_vs_zero_iter_ratio"] < 0.97, msg
    assert 0.8 < s["learned_vs_warm_iter_ratio"] < 1.2, msg


def test_learned_guess_3d_on_held_out_sphere_trajectory(L):
    """The 3D network (27-tap convolutions) trained on PPE solves of four
    seeded moving-sphere trajectories (32^3 mesh): the held-out loss falls
    below the warm start's, and every held-out PPE still reaches the
    tolerance from every start."""
    from paper_2404_17542_amd import configs, mcd as M
    n, ch = 32, (16, 32, 64)
    bc = configs.c4_moving_sphere(n=n).bc_pressure
    data = L.collect(range(1000, 1004), n, n_spin=6, n_save=30, log=lambda *_: None, flow="sphere")
    held = L.collect([2000], n, n_spin=6, n_save=6, log=lambda *_: None, flow="sphere")
    ctx = M.Context.from_case(configs.c4_moving_sphere(n=n))
    model = M.Model(ctx, ch)
    model.set_params(L.init_theta(ch, 0, dim=3))
    model.set_output_scale(L.output_scale(data, bc))
    before = L.eval_loss(model, held, bc)
    L.train(model, data, bc, epochs=8, lr=5e-4, seed=0, log=lambda *_: None)
    after = L.eval_loss(model, held, bc)
    modes = ("zero", "warm+jacobi", "learned", "warm")
    res = L.evaluate(model, [2000], n, n_spin=6, n_eval=6, modes=modes, log=lambda *_: None, flow="sphere")
    s = L.summarize(res)
    print({"loss_before": before, "loss_after": after, **s})
    assert before == pytest.approx(1.0)
    assert after < 0.7, after             # measured 0.34
    assert all(np.isfinite(v) for m in modes for v in res[m]["iters"]), s
    # the guess's initial residual is well below the warm start's (measured
    # 0.41 x); at 32^3 a solve takes only ~40 iterations, and the count is
    # about that of the warm start, which this test records but does not claim
    assert s["learned"]["mean_rel0"] < 0.7 * s["warm"]["mean_rel0"], s
