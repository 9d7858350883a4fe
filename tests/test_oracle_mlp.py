"""Pins for the FP64 cost-model oracle and the scheduling metrics."""
import numpy as np

from oracle import mlp, sched


def _data(n=200, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, mlp.N_IN))
    t = np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2] + 0.1 * rng.standard_normal(n)
    return X, t


def test_parameter_count():
    assert mlp.N_PARAMS == 5057


def test_gradient_matches_central_differences():
    X, t = _data(50)
    theta = mlp.init(3)
    mean, scale = X.mean(axis=0), X.std(axis=0)
    _, g = mlp.loss_grad(theta, X, t, mean, scale)
    rng = np.random.default_rng(1)
    h = 1e-6
    for p in rng.choice(mlp.N_PARAMS, 60, replace=False):
        e = np.zeros_like(theta)
        e[p] = h
        lp, _ = mlp.loss_grad(theta + e, X, t, mean, scale)
        lm, _ = mlp.loss_grad(theta - e, X, t, mean, scale)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[p]) <= 1e-6 * max(1.0, abs(fd)), p


def test_first_adam_step_closed_form():
    theta = np.zeros(4)
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    th, m, v = mlp.adam_step(theta, g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    np.testing.assert_allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_training_reduces_loss():
    X, t = _data(300)
    theta = mlp.init(5)
    mean, scale = X.mean(axis=0), X.std(axis=0)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0, _ = mlp.loss_grad(theta, X, t, mean, scale)
    for k in range(1, 301):
        _, g = mlp.loss_grad(theta, X, t, mean, scale)
        theta, m, v = mlp.adam_step(theta, g, m, v, k, lr=3e-3)
    l1, _ = mlp.loss_grad(theta, X, t, mean, scale)
    assert l1 < 0.2 * l0


def test_list_schedule_and_lpt():
    # two workers, costs 1,1,1,1,4: in this order the makespan is 6; LPT gives 4
    costs = np.array([1, 1, 1, 1, 4])
    busy = sched.list_schedule(costs, 2)
    assert busy.max() == 6 and abs(sched.load_balance(busy) - 8 / 12) < 1e-15
    order = sched.lpt_order(costs)
    assert list(order) == [4, 0, 1, 2, 3]
    busy = sched.list_schedule(costs[order], 2)
    assert busy.max() == 4 and sched.load_balance(busy) == 1.0


def test_class_order_hand_checked():
    # family 0: lower median 100 -> classes 0, 2, 0, 0; family 1: median 50
    # -> classes 0, -1, 2
    fam = np.array([0, 0, 0, 0, 1, 1, 1])
    pred = np.log(np.array([100.0, 400.0, 110.0, 95.0, 50.0, 25.0, 200.0])).astype(np.float32)
    assert list(sched.class_order(pred, fam)) == [1, 6, 0, 2, 3, 4, 5]
    # near-equal costs keep the given order entirely
    rng = np.random.default_rng(3)
    p = np.log(1000.0 * (1.0 + 0.3 * rng.random(50)))
    assert np.array_equal(sched.class_order(p, np.zeros(50, dtype=int)), np.arange(50))
    # the expensive item first: list scheduling on two workers
    costs = np.array([1.0, 1, 1, 1, 1, 1, 4])
    fam0 = np.zeros(7, dtype=int)
    assert sched.list_schedule(costs, 2).max() == 7
    assert sched.list_schedule(costs[sched.class_order(np.log(costs), fam0)], 2).max() == 5
    # a prediction half a class above the median rounds up, just below it down
    p = np.array([0.0, 0.0, 0.0, 0.5 * np.log(2.0) * (1 + 1e-12), 0.5 * np.log(2.0) * (1 - 1e-12)])
    assert list(sched.class_order(p, np.zeros(5, dtype=int))) == [3, 0, 1, 2, 4]
