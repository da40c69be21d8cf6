"""Host logic of the alignment drivers (CPU): the derivative-free pieces on
textbook functions, the eps schedule, and the pose error measure."""
import numpy as np
from scipy.spatial.transform import Rotation

from paper_1702_06813_amd import align as A


def test_nelder_mead_rosenbrock():
    """Rosenbrock's valley (the paper likens its cost to it): NM reaches (1, 1)."""
    f = lambda x: (1 - x[0]) ** 2 + 100 * (x[1] - x[0] ** 2) ** 2
    x, fx, ev = A.nelder_mead(f, np.array([-1.2, 1.0]), np.array([0.5, 0.5]), 2000, tol=1e-14)
    assert np.allclose(x, [1, 1], atol=1e-4) and fx < 1e-8


def test_coordinate_descent_separable_quadratic():
    c = np.array([0.3, -0.2, 0.05, 0.1, -0.4, 0.25])
    f = lambda x: float(np.sum((x - c) ** 2))
    x, fx, ev = A.coordinate_descent(f, np.zeros(6), f(np.zeros(6)), np.full(6, 0.1), 5000, min_step=1e-6)
    assert np.allclose(x, c, atol=1e-5)


def test_hybrid_on_quantized_cost_within_budget():
    """A piecewise-constant cost (integer counts, like Table I's E): the
    hybrid optimizer gets within the quantization of the minimum using at
    most its evaluation budget."""
    c = np.array([0.04, -0.03, 0.02, 0.03, -0.02, 0.01])
    calls = []
    def f(x):
        calls.append(1)
        return float(np.floor(2e4 * np.sum((x - c) ** 2)))
    x, fx, ev = A.hybrid_minimize(f, budget=700)
    assert ev == len(calls) <= 700
    assert np.sum((x - c) ** 2) < 3e-4


def test_eps_schedule():
    e = A.eps_schedule(20, 0.5, 0.1)
    assert len(e) == 20 and abs(e[0] - 0.5) < 1e-12 and abs(e[-1] - 0.1) < 1e-12
    assert all(a > b for a, b in zip(e, e[1:]))
    assert A.eps_schedule(1) == [0.1]


def test_pose_errors():
    T = np.zeros((3, 4)); T[:, :3] = np.eye(3)
    T2 = T.copy(); T2[:, :3] = Rotation.from_rotvec([0, 0, 0.1]).as_matrix(); T2[:, 3] = [0.03, 0.04, 0]
    dt, ang = A.pose_errors(T2, T)
    assert abs(dt[0] - 0.05) < 1e-12 and abs(ang[0] - 0.1) < 1e-9


def test_lockstep_equals_one_at_a_time():
    """Driving several hybrid optimizers together (one batched evaluation per
    round) gives each exactly the result it reaches alone, in as many rounds
    as the longest instance needs."""
    rng = np.random.default_rng(4)
    cs = [rng.normal(scale=0.03, size=6) for _ in range(5)]
    fs = [lambda x, c=c: float(np.floor(2e4 * np.sum((x - c) ** 2))) for c in cs]
    alone = [A.hybrid_minimize(f, budget=300) for f in fs]
    res, rounds = A.lockstep([A._hybrid(budget=300) for _ in fs],
                             lambda ks, xs: [fs[k](x) for k, x in zip(ks, xs)])
    for (x1, f1, e1), (x2, f2, e2) in zip(alone, res):
        np.testing.assert_array_equal(x1, x2)
        assert f1 == f2 and e1 == e2
    assert rounds == max(e for _, _, e in alone)


# ---------------------------------------------------------------- Adam (oracle pins)

def test_adam_first_step_is_lr_times_sign(oracle_mod):
    """With zero moments, bias correction makes the first step
    -lr g / (|g| + 1e-12) per component: -lr sign(g) up to the guard."""
    O = oracle_mod
    rng = np.random.default_rng(0)
    g = rng.normal(size=6) * 10.0 ** rng.uniform(-3, 3, 6)
    d, m, v = O.adam_step(g, np.zeros(6), np.zeros(6), 1, lr=0.01)
    np.testing.assert_allclose(d, -0.01 * g / (np.abs(g) + 1e-12), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)


def test_adam_constant_gradient_keeps_unit_steps(oracle_mod):
    """A constant gradient gives m_hat = g and v_hat = g^2 at every step, so
    every step is -lr g / (|g| + 1e-12): a wrong bias correction drifts from it."""
    O = oracle_mod
    g = np.array([3.0, -0.5, 1e-3, -2e2, 7.0, 0.25])
    m, v = np.zeros(6), np.zeros(6)
    for k in range(1, 40):
        d, m, v = O.adam_step(g, m, v, k, lr=0.05, beta1=0.8, beta2=0.95)
        np.testing.assert_allclose(d, -0.05 * g / (np.abs(g) + 1e-12), rtol=1e-12)


def test_adam_converges_on_quadratic_bowl(oracle_mod):
    """Adam on f(x) = 1/2 (x - c)^T A (x - c) with an ill-conditioned A reaches
    the minimum c to within a fraction of the step size."""
    O = oracle_mod
    A = np.diag([100.0, 10.0, 1.0, 0.1, 3.0, 30.0])
    c = np.array([0.3, -0.2, 0.1, 0.05, -0.4, 0.25])
    x = np.zeros(6)
    m, v = np.zeros(6), np.zeros(6)
    lr = 0.01
    for k in range(1, 3001):
        lr_k = lr * (0.999 ** k)
        d, m, v = O.adam_step(A @ (x - c), m, v, k, lr=lr_k)
        x = x + d
    assert np.abs(x - c).max() < 1e-3, x - c


# ---------------------------------------------------------------- speculative batches of the paper's optimizer

def _cases():
    rng = np.random.default_rng(7)
    cs = [rng.normal(scale=0.03, size=6) for _ in range(4)]
    fs = [lambda x, c=c: float(np.floor(2e4 * np.sum((x - c) ** 2))) for c in cs]          # plateaus like E(X)
    fs.append(lambda x: float(np.sum(100 * (x[1:] - x[:-1] ** 2) ** 2 + (1 - x[:-1]) ** 2)))  # Rosenbrock
    fs.append(lambda x: float(np.floor(50 * np.sum(np.abs(x - 0.01)))))                       # coarse plateaus
    fs.append(lambda x: 0.0)                                                                   # flat: zero gradient
    return fs


def test_speculative_batches_reproduce_the_sequential_optimizer():
    """The batch form of the hybrid optimizer (stencil, line search, simplex,
    Nelder-Mead candidates and coordinate-descent probes requested together)
    ends at exactly the point, cost and evaluation count of the one-point
    form, for costs with plateaus, a smooth valley and a flat cost, under
    budgets that stop it in each phase; it needs far fewer batches than
    evaluations."""
    for f in _cases():
        for budget in (30, 57, 120, 333, 700):
            x1, f1, e1 = A.hybrid_minimize(f, budget=budget)
            x2, f2, e2, nb = A.hybrid_minimize_batched(lambda xs: [f(x) for x in xs], budget=budget)
            np.testing.assert_array_equal(x1, x2)
            assert f1 == f2 and e1 == e2, (budget, e1, e2)
            assert nb <= e1
    f = _cases()[0]
    _, _, ev, nb = A.hybrid_minimize_batched(lambda xs: [f(x) for x in xs], budget=700)
    assert nb < ev / 3, (nb, ev)


def test_lockstep_of_speculative_batches_equals_one_at_a_time():
    fs = _cases()[:5]
    alone = [A.hybrid_minimize(f, budget=300) for f in fs]
    res, rounds = A.lockstep_batches([A._hybrid_b(budget=300) for _ in fs],
                                     lambda ks, bs: [[fs[k](x) for x in b] for k, b in zip(ks, bs)])
    for (x1, f1, e1), (x2, f2, e2) in zip(alone, res):
        np.testing.assert_array_equal(x1, x2)
        assert f1 == f2 and e1 == e2
    assert rounds < max(e for _, _, e in alone)
