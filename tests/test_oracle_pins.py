"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Each test names the passage it rests on.  None of them re-types the oracle's
formulas: they check defining properties (a projection lies on its
hyperplane), exact rational arithmetic, closed forms of a structured system,
inequalities that follow from feasibility of a known point, invariances, and
exhaustive geometry for n <= 3.
"""
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import brute

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# ---------------------------------------------------------------- P1: one inequality = orthogonal projection
@pytest.mark.parametrize("seed", range(5))
def test_single_row_avg_step_is_orthogonal_projection(oracle_lib, seed):
    """Section 2: pi_H(x) = x - rho_H(x) lies on H and x - pi_H(x) is parallel to a.

    With one row, h = 1 and phi = rho+ (eq. 8), so Algorithm 1 (lambda = 1)
    maps a violating x to its projection onto H.
    """
    rng = np.random.default_rng(seed)
    n = 7
    a = rng.normal(size=(1, n))
    x = rng.normal(size=n)
    b = np.array([a[0] @ x - 1.5])          # x violates the row by 1.5
    s = oracle_lib.sweep(a, "f64", b, x)
    assert s.h == 1
    x1, st = oracle_lib.step(s.y, s.h, 1, 1.0, x)
    assert st == 0
    # on the hyperplane
    assert abs(a[0] @ x1 - b[0]) <= 1e-13 * (np.abs(a[0]) @ np.abs(x1) + abs(b[0]))
    # displacement parallel to a: the component orthogonal to a vanishes
    d = x1 - x
    u = a[0] / np.linalg.norm(a[0])
    assert np.linalg.norm(d - (d @ u) * u) <= 1e-13 * np.linalg.norm(d)
    # distance moved equals the distance to the hyperplane, 1.5/||a||
    assert np.linalg.norm(d) == pytest.approx(1.5 / np.linalg.norm(a[0]), rel=1e-14)


@pytest.mark.parametrize("lam", [0.25, 1.0, 3.0])
def test_single_row_fixed_step_has_length_lambda(oracle_lib, lam):
    """Eq. 12: the ModAP step psi always has length lambda; at lambda = r/||a|| it is the projection."""
    rng = np.random.default_rng(11)
    n = 5
    a = rng.normal(size=(1, n))
    x = rng.normal(size=n)
    b = np.array([a[0] @ x - 0.7])
    s = oracle_lib.sweep(a, "f64", b, x)
    x1, _ = oracle_lib.step(s.y, s.h, 0, lam, x)
    assert np.linalg.norm(x1 - x) == pytest.approx(lam, rel=1e-14)
    # direction -a/||a||
    assert np.allclose((x - x1) / lam, a[0] / np.linalg.norm(a[0]), atol=1e-14)
    lam_proj = 0.7 / np.linalg.norm(a[0])
    x2, _ = oracle_lib.step(s.y, s.h, 0, lam_proj, x)
    assert abs(a[0] @ x2 - b[0]) <= 1e-13 * (1 + abs(b[0]))


# ---------------------------------------------------------------- P2: a feasible point is a fixed point
def test_feasible_point_is_fixed(oracle_lib):
    """Eq. 7: rho+ is non-zero iff x violates row i; a feasible x gives y = 0, h = 0, a stop."""
    sys_ = W.gaussian(40, 90, seed=3, dtype="f64")
    s = oracle_lib.sweep(sys_.A, "f64", sys_.b, sys_.z)
    assert s.h == 0 and s.dmax == 0.0 and np.all(s.y == 0.0)
    assert np.all(s.r < 0)
    res = oracle_lib.solve(sys_.A, "f64", sys_.b, sys_.z, lam=1.0, eps=1e-6)
    assert res.status == 0 and res.iters == 0
    assert np.array_equal(res.x, sys_.z)


# ---------------------------------------------------------------- P3: closed form for the box-plus-sum system
def _box_sum_closed_form(x, upper=200.0):
    n = x.size
    agg = x.sum() - upper * (n - 1)
    y = np.maximum(x - upper, 0) - np.maximum(-x, 0) + max(agg, 0.0) / n
    h = int(np.sum(x > upper) + np.sum(x < 0) + (agg > 0))
    d = [np.max(np.maximum(x - upper, 0), initial=0.0), np.max(np.maximum(-x, 0), initial=0.0),
         max(agg, 0.0) / math.sqrt(n)]
    return y, h, max(d)


@pytest.mark.parametrize("seed", range(6))
def test_box_sum_sweep_matches_closed_form(oracle_lib, seed):
    """Rows e_j (b = 200), -e_j (b = 0), 1 (b = 200(n-1)): each positive slice has a closed form."""
    n = 64
    sys_ = W.box_sum(n, seed=seed)
    rng = np.random.default_rng(100 + seed)
    x = [sys_.x0, rng.uniform(-50, 250, n), np.full(n, 100.0), rng.uniform(150, 260, n)][seed % 4]
    s = oracle_lib.sweep(sys_.A, "f64", sys_.b, x)
    y, h, dmax = _box_sum_closed_form(x)
    assert s.h == h
    np.testing.assert_allclose(s.y, y, rtol=1e-15, atol=1e-12)
    assert s.dmax == pytest.approx(dmax, rel=1e-15, abs=1e-12)
    assert s.binf == 200.0 * (n - 1)


# ---------------------------------------------------------------- exact rational sweep (brute force)
@pytest.mark.parametrize("seed", range(8))
def test_sweep_equals_exact_rational_sweep(oracle_lib, seed):
    """One sweep from its plain definition (eqs. 7, 8, 10) in exact rationals.

    Dyadic inputs (k/8) make every FP64 input exact, so the only error left in
    the oracle is its final rounding.
    """
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 6))
    m = int(rng.integers(1, 10))
    A = rng.integers(-16, 17, size=(m, n)) / 8.0
    A[np.all(A == 0, axis=1), 0] = 1.0
    x = rng.integers(-40, 41, size=n) / 8.0
    b = rng.integers(-30, 31, size=m) / 8.0
    s = oracle_lib.sweep(A, "f64", b, x)
    r, h, y, d2 = brute.exact_sweep(A, b, x)
    np.testing.assert_array_equal(s.r, np.array([float(v) for v in r]))  # dyadic: exact
    assert s.h == h
    yref = np.array([float(v) for v in y])
    np.testing.assert_allclose(s.y, yref, rtol=2.3e-16, atol=1e-300)
    dref = math.sqrt(float(max(d2))) if d2 else 0.0
    assert s.dmax == pytest.approx(dref, rel=4.5e-16)


@pytest.mark.parametrize("seed", range(8))
def test_rounding_scale_equals_exact_rational_scale(oracle_lib, seed):
    """The rounding-error scale t_i = sum_j |a_ij x_j| + |b_i| that every GPU
    tolerance is measured on, against its definition in exact rationals.
    Dyadic inputs of mixed signs (k/8, b_i of both signs) make every term and
    partial sum exact in FP64, so t must match exactly: a dropped |b_i|, a
    signed instead of an absolute product or a missing term would not."""
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 7))
    m = int(rng.integers(2, 12))
    A = rng.integers(-16, 17, size=(m, n)) / 8.0
    A[np.all(A == 0, axis=1), 0] = -1.0
    x = rng.integers(-40, 41, size=n) / 8.0
    b = rng.integers(-30, 31, size=m) / 8.0
    b[0] = -abs(b[0]) - 0.5                 # at least one negative right-hand side
    s = oracle_lib.sweep(A, "f64", b, x)
    t = brute.exact_scale(A, b, x)
    np.testing.assert_array_equal(s.t, np.array([float(v) for v in t]))
    # t bounds the residual (triangle inequality), with equality only when all
    # terms of row i have one sign
    assert np.all(np.abs(s.r) <= s.t)


def test_rounding_scale_of_stored_rows(oracle_lib):
    """t is taken on the stored (widened) rows: for BF16 storage the scale of
    a row whose entries were rounded is that of the rounded entries."""
    A64 = np.array([[1.0 + 2.0 ** -9, -3.0], [0.5, 0.25]])   # 1 + 2^-9 is not a BF16 value
    Ab = W.encode(A64, "bf16")
    x = np.array([2.0, -1.0])
    b = np.array([-1.0, 0.75])
    s = oracle_lib.sweep(Ab, "bf16", b, x)
    Aw = W.stored_to_f64(Ab, "bf16")
    assert Aw[0, 0] != A64[0, 0]
    t = brute.exact_scale(Aw, b, x)
    np.testing.assert_array_equal(s.t, np.array([float(v) for v in t]))


def test_storage_widening_is_exact(oracle_lib):
    """BF16 is the top half of a binary32: the oracle's widening agrees with an
    independent bit-level widening, so the same stored bytes give the same sweep."""
    sys_ = W.gaussian(33, 70, seed=5, dtype="bf16")
    A64 = W.bf16_bits_to_f64(sys_.A)
    x = np.random.default_rng(0).normal(size=33)
    s16 = oracle_lib.sweep(sys_.A, "bf16", sys_.b, x)
    s64 = oracle_lib.sweep(A64, "f64", sys_.b, x)
    np.testing.assert_array_equal(s16.r, s64.r)
    np.testing.assert_array_equal(s16.y, s64.y)
    sys32 = W.gaussian(33, 70, seed=5, dtype="f32")
    s32 = oracle_lib.sweep(sys32.A, "f32", sys32.b, x)
    s3264 = oracle_lib.sweep(sys32.A.astype(np.float64), "f64", sys32.b, x)
    np.testing.assert_array_equal(s32.y, s3264.y)


def test_bf16_encoding_round_to_nearest_even():
    """RNE on the 16 dropped bits, including the tie cases."""
    vals = np.array([1.0, 1.0 + 2**-8, 1.0 + 2**-7 + 2**-8, -3.5, 1.0 + 2**-8 + 2**-20], dtype=np.float32)
    bits = W.f32_to_bf16_bits(vals)
    back = W.bf16_bits_to_f64(bits)
    # 1 + 2^-8 is a tie -> even (1.0); 1 + 2^-7 + 2^-8 is a tie -> even (1 + 2^-6)
    np.testing.assert_array_equal(back, [1.0, 1.0, 1.0 + 2**-6, -3.5, 1.0 + 2**-7])


# ---------------------------------------------------------------- P4: Fejer inequality with a known feasible point
@pytest.mark.parametrize("seed", range(4))
def test_fejer_inequality_and_avg_step_monotone(oracle_lib, seed):
    """Section 2 (Algorithm 1 is an M-Fejer mapping): from a_i.z <= b_i,
    <x - z, y> >= sum_V r_i^2/||a_i||^2, and the relaxed step with lambda in
    (0, 2) satisfies ||x' - z||^2 <= ||x - z||^2 - lambda(2 - lambda)||phi||^2."""
    sys_ = W.gaussian(24, 60, seed=seed, dtype="f64")
    x = sys_.z + np.random.default_rng(seed).normal(scale=3.0, size=24)
    s = oracle_lib.sweep(sys_.A, "f64", sys_.b, x)
    assert s.h > 0
    viol = s.r > 0
    lhs = (x - sys_.z) @ s.y
    rhs = np.sum(s.r[viol] ** 2 / s.nu[viol])
    assert lhs >= rhs * (1 - 1e-12)
    for lam in (0.5, 1.0, 1.5):
        x1, _ = oracle_lib.step(s.y, s.h, 1, lam, x)
        phi = s.y / s.h
        before = np.sum((x - sys_.z) ** 2)
        after = np.sum((x1 - sys_.z) ** 2)
        assert after <= before - lam * (2 - lam) * (phi @ phi) + 1e-9 * before


# ---------------------------------------------------------------- P5: finite termination of ModAP
def test_modap_finite_termination_bound(oracle_lib):
    """Section 2 claims a finite number of steps for a fixed polytope.  If the
    ball B(c, rho) lies in M and lambda < 2 rho, then <x - c, y/||y||> >= rho and
    each ModAP step decreases ||x - c||^2 by at least lambda(2 rho - lambda)."""
    n = 16
    sys_ = W.box_sum(n, seed=4)
    c = np.full(n, 100.0)
    rho, lam = 100.0, 1.0
    res = oracle_lib.solve(sys_.A, "f64", sys_.b, sys_.x0, lam=lam, eps=1e-6,
                           rule=0, max_steps=20000, x_trace=True)
    assert res.status == 0
    bound = np.sum((sys_.x0 - c) ** 2) / (lam * (2 * rho - lam))
    assert res.iters <= bound
    dist2 = np.sum((res.x_trace - c) ** 2, axis=1)
    assert np.all(np.diff(dist2) <= -lam * (2 * rho - lam) * (1 - 1e-9))
    # the final point is eps-feasible by direct evaluation
    viol = (sys_.A @ res.x - sys_.b) / np.linalg.norm(sys_.A, axis=1)
    assert viol.max() <= 1e-6 * np.abs(sys_.b).max()


# ---------------------------------------------------------------- P6: brute force, n = 2 and 3
def _random_polytope(rng, n, m):
    """A bounded polytope: a box of half-width 2 around the origin plus random cuts
    that keep a ball of radius 0.5 around the origin."""
    rows, rhs = [], []
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        rows += [e, -e]
        rhs += [2.0, 2.0]
    for _ in range(m):
        a = rng.normal(size=n)
        rows.append(a)
        rhs.append(np.linalg.norm(a) * rng.uniform(0.5, 1.5))
    return np.array(rows), np.array(rhs)


@pytest.mark.parametrize("n,seed", [(2, 0), (2, 1), (3, 2), (3, 3)])
def test_brute_force_fejer_distance_and_feasible_end(oracle_lib, n, seed):
    """d(x_k, M) never increases under Algorithm 1 (Fejer, section 2), and the
    final points of both step rules are eps-feasible (eq. 10)."""
    rng = np.random.default_rng(seed)
    A, b = _random_polytope(rng, n, 4)
    assert len(brute.vertices(A, b)) >= n + 1          # non-empty, full-dimensional
    x0 = rng.normal(scale=6.0, size=n)
    eps = 1e-7
    res = oracle_lib.solve(A, "f64", b, x0, lam=1.0, eps=eps, eps_relative=False, rule=1,
                           max_steps=200000, x_trace=True)
    assert res.status == 0
    dists = [brute.project(A, b, xk)[1] for xk in res.x_trace[:: max(1, len(res.x_trace) // 200)]]
    assert np.all(np.diff(dists) <= 1e-12)
    for rule, lam in ((0, 0.05), (1, 1.0)):
        r2 = oracle_lib.solve(A, "f64", b, x0, lam=lam, eps=eps, eps_relative=False, rule=rule,
                              max_steps=200000)
        assert r2.status == 0
        viol = np.maximum(A @ r2.x - b, 0) / np.linalg.norm(A, axis=1)
        assert viol.max() <= eps


def _narrow_wedge(delta):
    # thin triangle with its vertex at the origin: x2 <= delta x1, -x2 <= delta x1, x1 <= 1
    A = np.array([[-delta, 1.0], [-delta, -1.0], [1.0, 0.0]])
    b = np.array([0.0, 0.0, 1.0])
    return A, b


def test_narrow_vertex_slows_fejer_steps_not_fixed_steps(oracle_lib):
    """Section 2 (Fig. 2 discussion): near a narrow vertex the Fejer steps of
    Algorithm 1 crawl towards M, while ModAP's fixed-length step enters it."""
    A, b = _narrow_wedge(0.02)
    x0 = np.array([-1.0, 0.0])
    avg = oracle_lib.solve(A, "f64", b, x0, lam=1.0, eps=1e-7, eps_relative=False, rule=1,
                           max_steps=400000)
    fix = oracle_lib.solve(A, "f64", b, x0, lam=0.3, eps=1e-7, eps_relative=False, rule=0,
                           max_steps=400000)
    assert avg.status == 0 and fix.status == 0
    assert fix.iters <= 5
    assert avg.iters > 1000 * fix.iters


def test_moving_narrow_vertex_is_caught_only_by_fixed_steps(oracle_lib):
    """Section 2: when the polytope moves, the Fejer process of Algorithm 1
    never reaches eps-feasibility, while the fixed-length ModAP step catches up
    whenever lambda exceeds the displacement per iteration."""
    A, b = _narrow_wedge(0.02)
    x0 = np.array([-1.0, 0.0])
    V = np.tile([1e-3, 0.0], (20000, 1))            # translate M along +x1 each iteration
    avg = oracle_lib.solve(A, "f64", b, x0, lam=1.0, eps=1e-7, eps_relative=False, rule=1,
                           max_steps=20000, V=V)
    fix = oracle_lib.solve(A, "f64", b, x0, lam=0.3, eps=1e-7, eps_relative=False, rule=0,
                           max_steps=20000, V=V)
    assert avg.status == 1                           # step limit, never eps-feasible
    assert fix.status == 0 and fix.iters < 20


# ---------------------------------------------------------------- P7, P8: invariances
def test_translation_invariance(oracle_lib):
    """Translating M by v (b -> b + A v) and x by v leaves every positive slice unchanged."""
    sys_ = W.gaussian(30, 80, seed=9, dtype="f64")
    rng = np.random.default_rng(9)
    x = rng.normal(size=30) * 2
    v = rng.normal(size=30)
    s0 = oracle_lib.sweep(sys_.A, "f64", sys_.b, x)
    b1 = oracle_lib.translate(sys_.A, "f64", sys_.b, v)
    s1 = oracle_lib.sweep(sys_.A, "f64", b1, x + v)
    np.testing.assert_allclose(s1.r, s0.r, atol=1e-13 * np.max(s0.t))
    assert s1.h == s0.h
    np.testing.assert_allclose(s1.y, s0.y, rtol=1e-12, atol=1e-13)
    assert s1.dmax == pytest.approx(s0.dmax, rel=1e-12)


def test_row_scaling_and_permutation_invariance(oracle_lib):
    """Eq. 7 is unchanged by (a_i, b_i) -> (c a_i, c b_i) for c > 0, and the
    Reduce(+) does not depend on the order of the list."""
    sys_ = W.gaussian(20, 50, seed=2, dtype="f64")
    rng = np.random.default_rng(2)
    x = rng.normal(size=20) * 2
    c = 2.0 ** rng.integers(-3, 4, size=50)         # powers of two: exact scaling
    perm = rng.permutation(50)
    s0 = oracle_lib.sweep(sys_.A, "f64", sys_.b, x)
    s1 = oracle_lib.sweep((sys_.A * c[:, None])[perm], "f64", (sys_.b * c)[perm], x)
    assert s1.h == s0.h
    np.testing.assert_allclose(s1.y, s0.y, rtol=1e-14, atol=1e-15)
    assert s1.dmax == pytest.approx(s0.dmax, rel=1e-15)
    np.testing.assert_allclose(s1.r, (s0.r * c)[perm], rtol=1e-15, atol=1e-15)


def test_zero_row_is_reported(oracle_lib):
    """Section 2 assumes a_i != 0 for every row."""
    A = np.array([[1.0, 2.0], [0.0, 0.0], [1.0, -1.0]])
    nu, bad = oracle_lib.norms(A, "f64")
    assert bad == 1
    res = oracle_lib.solve(A, "f64", np.zeros(3), np.ones(2))
    assert res.status == 3


def test_row_replacement(oracle_lib):
    """Coefficients and right-hand sides may change during the computation (section 1)."""
    sys_ = W.gaussian(16, 40, seed=1, dtype="f32")
    idx, rows, bb = W.replacement_rows(sys_, 4, seed=1)
    A2, b2 = oracle_lib.replace_rows(sys_.A, "f32", sys_.b, idx, rows, bb)
    np.testing.assert_array_equal(A2[idx], rows)
    np.testing.assert_array_equal(b2[idx], bb)
    keep = np.setdiff1d(np.arange(40), idx)
    np.testing.assert_array_equal(A2[keep], sys_.A[keep])
    # the hidden point stays strictly feasible for the new rows
    assert np.all(A2.astype(np.float64) @ sys_.z < b2)


# ---------------------------------------------------------------- P10: printed rate arithmetic
def test_paper_catchup_rate_arithmetic():
    """Section 5: the total displacement rate is the length of the vector that
    adds r units/s to each of the n coordinates, sqrt(n r^2)."""
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_catchup_rates.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) == 6
    for n, K, r, total, _ in rows:
        n, r, total = int(n), int(r), int(total)
        assert round(math.sqrt(n * r * r)) == total
        V = W.line_drift(n, 1, r)
        assert round(float(np.linalg.norm(V[0]))) == total


def test_point_on_hyperplane_is_not_violated(oracle_lib):
    """Eq. 7: max(<a_i,x> - b_i, 0) = 0 on H_i, so a row met with equality adds
    no term and is not counted in h (eq. 8)."""
    A = np.array([[1.0, 0.0], [0.0, 1.0], [1.0, 1.0], [-1.0, 0.0]])
    b = np.array([1.0, 2.0, 3.0, 5.0])
    x = np.array([1.0, 2.0])                     # rows 0, 1, 2 hold with equality
    s = oracle_lib.sweep(A, "f64", b, x)
    assert s.h == 0 and s.dmax == 0.0 and np.all(s.y == 0.0)
    x2 = np.array([1.0, 2.5])                    # now rows 1, 2 are violated, row 0 is tight
    s2 = oracle_lib.sweep(A, "f64", b, x2)
    assert s2.h == 2


def test_relative_tolerance_uses_current_rhs_max(oracle_lib):
    """Reading of eq. 10 used for the configurations: eps_abs = eps * max_i |b_i|
    of the current data.  A point 0.5 outside a row with max|b| = 1000 is
    accepted at eps = 1e-3 (eps_abs = 1) but not at an absolute 1e-3."""
    A = np.array([[1.0, 0.0], [0.0, 1.0]])
    b = np.array([1000.0, 0.0])
    x = np.array([0.0, 0.5])
    rel = oracle_lib.solve(A, "f64", b, x, lam=0.1, eps=1e-3, eps_relative=True, rule=0)
    ab = oracle_lib.solve(A, "f64", b, x, lam=0.1, eps=1e-3, eps_relative=False, rule=0)
    assert rel.status == 0 and rel.iters == 0
    assert ab.status == 0 and ab.iters == 5
    # translation changes max|b| and with it the threshold
    V = np.array([[0.0, -2000.0]])
    moved = oracle_lib.solve(A, "f64", b, np.array([0.0, 1.5]), lam=1.0, eps=1e-3,
                             eps_relative=True, rule=0, max_steps=1, V=V)
    # after one step (x2 = 0.5) and the translation b2 -> -2000: max|b| = 2000,
    # the point is 2000.5 outside row 2: not accepted
    assert moved.status == 1
