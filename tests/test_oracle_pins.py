"""Pins of the FP64 CPU oracle against facts fixed by the paper and by the
mathematics (closed forms, invariants, exact rational brute force, a library
QR and a library distance routine), never against the oracle itself.

Each test names the part of the method it pins:
  evaluation  -- r_ij = ||P^T s_ij||, its min and argmin (Sec. 4, objective;
                 Algorithm 1, argmin step)
  update      -- argmax / MGS / shift (Sec. 4 prose; Algorithm 1)
  loop        -- Algorithm 1's iteration
  soft-min    -- the differentiable surrogate and its gradient
"""
from fractions import Fraction
from pathlib import Path

import numpy as np
import pytest
from scipy.spatial.distance import pdist

import oracle
from oracle import tiny_exact
import sap_inputs

GOLDEN = Path(__file__).parent / "golden"


def _pairs(N):
    return [(i, j) for i in range(N) for j in range(i + 1, N)]


# ---------------------------------------------------------------- evaluation

def test_projection_bound_all_pairs():
    """P1: a projection cannot lengthen a unit vector, 0 <= r <= 1 (Sec. 3.3)."""
    w = sap_inputs.make("trig10", N=120)
    r, _ = oracle.all_r(w.X, w.P0)
    assert np.all(r >= 0.0) and np.all(r <= 1.0 + 1e-15)
    m = oracle.min_secant(w.X, w.P0)
    assert m["r_max"] <= 1.0 + 1e-15 and m["n_pairs"] == len(r)


def test_k_equals_n_gives_one():
    """P2: with k = n the projection is the identity on R^n, every r = 1."""
    rng = np.random.default_rng(7)
    X = rng.standard_normal((40, 6))
    P = sap_inputs.random_orthonormal(rng, 6, 6)
    m = oracle.min_secant(X, P)
    assert abs(m["r_min"] - 1.0) < 1e-14 and abs(m["r_max"] - 1.0) < 1e-14


def test_affine_plane_data_gives_one():
    """P3: data on an affine k-plane with P spanning that plane: every secant
    lies in span(P), so min = 1, and the update leaves span(P) unchanged."""
    rng = np.random.default_rng(11)
    n, k = 9, 3
    A = sap_inputs.random_orthonormal(rng, n, k)
    Z = rng.standard_normal((50, k))
    b = rng.standard_normal(n)
    X = Z @ A.T + b[None, :]
    Q = sap_inputs.random_orthonormal(rng, k, k)
    P = A @ Q
    m = oracle.min_secant(X, P)
    assert abs(m["r_min"] - 1.0) < 1e-13
    s, _ = oracle.unit_secant(X, m["i"], m["j"])
    P2, _ = oracle.step(P, s, 0.01)
    assert np.abs(P2 @ P2.T - A @ A.T).max() < 1e-13


def test_naive_projection_trig_curve_bound():
    """P4 (Sec. 5 curve): for P = [e1, e2, e3] every r >= 1/sqrt(55), and the
    bound is approached by close pairs near t in {0, pi/2, pi, 3pi/2}.  The
    printed value of the paper lies below the bound (see the golden file)."""
    gold = dict(l.split() for l in (GOLDEN / "trig_curve_sec5.txt").read_text().splitlines()
                if l and not l.startswith("#"))
    bound = float(gold["bound_naive"])
    assert abs(bound - 1.0 / np.sqrt(55.0)) < 1e-16
    assert float(gold["naive"]) < bound       # the paper's number is not reachable
    P = np.zeros((10, 3)); P[0, 0] = P[1, 1] = P[2, 2] = 1.0
    w = sap_inputs.make("trig10", N=200)
    m = oracle.min_secant(w.X, P)
    assert m["r_min"] >= bound - 1e-15
    # dense samples near t = 0 from both sides approach the infimum closely
    t = np.concatenate([np.linspace(-0.02, 0.02, 41), [np.pi / 2 + 0.001, np.pi / 2 - 0.001]])
    h = np.arange(1, 6)
    X = np.empty((t.size, 10)); X[:, 0::2] = np.cos(np.outer(t, h)); X[:, 1::2] = np.sin(np.outer(t, h))
    m2 = oracle.min_secant(X, P)
    assert bound - 1e-15 <= m2["r_min"] < bound + 2e-4


def test_against_library_distances():
    """The evaluation by explicit unit secants agrees with an independent
    route: project first, then r = ||y_i - y_j|| / ||x_i - x_j|| with scipy's
    pdist, on well-separated data (no cancellation at this scale)."""
    for name, N in (("trig10", 150), ("trig64", 90), ("hyper", 80)):
        w = sap_inputs.make(name, N=N)
        X = w.X.astype(np.float64)
        r, d = oracle.all_r(X, w.P0)
        r_lib = pdist(X @ w.P0) / pdist(X)
        assert np.allclose(d, pdist(X), rtol=1e-14, atol=0)
        assert np.max(np.abs(r - r_lib)) < 1e-11
        m = oracle.min_secant(X, w.P0)
        q = int(np.argmin(r_lib))
        gap = np.partition(r_lib, 1)[1] - r_lib[q]
        if gap > 1e-9:
            assert _pairs(N)[q] == (m["i"], m["j"])
        assert abs(m["r_min"] - r_lib.min()) < 1e-11


def test_basis_translation_scale_permutation_invariance():
    """P5: (min, argmin) depend on span(P) only, and are invariant to
    translating or scaling X; permuting points permutes the argmin."""
    w = sap_inputs.make("trig64", N=70)
    X = w.X.astype(np.float64)
    m = oracle.min_secant(X, w.P0)
    rng = np.random.default_rng(3)
    Q = sap_inputs.random_orthonormal(rng, w.k, w.k)
    for X2, P2 in ((X, w.P0 @ Q), (X + 3.5, w.P0), (X * 2.0, w.P0)):
        m2 = oracle.min_secant(X2, P2)
        assert abs(m2["r_min"] - m["r_min"]) < 1e-13
        assert (m2["i"], m2["j"]) == (m["i"], m["j"])
    perm = rng.permutation(X.shape[0])
    m3 = oracle.min_secant(X[perm], w.P0)
    inv = np.argsort(perm)
    assert sorted((inv[m["i"]], inv[m["j"]])) == [m3["i"], m3["j"]]


def test_exact_rational_brute_force_and_ties():
    """P10: on tiny rational inputs the FP64 argmin equals the exact-rational
    lexicographic (r, i, j) argmin, including constructed exact ties."""
    # parallel secants (identical unit secant, identical r): tie by (i, j)
    X = [[0, 0, 0], [1, 0, 0], [2, 0, 0], [0, 1, 0], [0, 0, 3], [5, 2, 0]]
    P = [[0, 0], [1, 0], [0, 1]]                   # e2, e3: r = 0 for x-axis secants
    v, i, j, allv = tiny_exact.min_exact(X, P)
    assert v == 0 and (i, j) == (0, 1)
    assert tiny_exact.is_orthonormal_exact(P)
    m = oracle.min_secant(np.array(X, float), np.array(P, float))
    assert (m["i"], m["j"]) == (i, j) and m["r_min"] == 0.0
    # the runner-up is the next tied pair in lexicographic order
    assert (m["i2"], m["j2"]) == allv[1][1:]
    # rational rotation (3/5, 4/5) and random small-integer points
    rng = np.random.default_rng(5)
    Pq = [[Fraction(3, 5), Fraction(0)], [Fraction(4, 5), Fraction(0)], [Fraction(0), Fraction(1)],
          [Fraction(0), Fraction(0)]]
    assert tiny_exact.is_orthonormal_exact(Pq)
    Pf = np.array([[float(a) for a in row] for row in Pq])
    for _ in range(25):
        Xi = rng.integers(-3, 4, size=(7, 4))
        v, i, j, allv = tiny_exact.min_exact(Xi.tolist(), Pq)
        m = oracle.min_secant(Xi.astype(float), Pf)
        assert abs(m["r_min"] - float(v) ** 0.5) < 1e-15
        # the exact argmin must win unless an exact tie is broken by (i, j),
        # in which case both agree on the lexicographic pick
        assert (m["i"], m["j"]) == (i, j) or (abs(float(allv[1][0]) - float(v)) < 1e-15)


def test_duplicates_and_length_threshold():
    """Duplicates have no unit secant; Sec. 7 drops secants shorter than l."""
    X = np.array([[0.0, 0.0], [0.0, 0.0], [1.0, 0.0], [0.0, 3.0]])
    P = np.array([[1.0], [0.0]])
    m = oracle.min_secant(X, P)
    assert m["n_pairs"] == 5 and m["n_dropped"] == 1
    m = oracle.min_secant(X, P, min_len=1.5)      # drops d=0 and the two d=1 pairs
    assert m["n_pairs"] == 3 and m["n_dropped"] == 3
    v, i, j, _ = tiny_exact.min_exact(X.tolist(), P.tolist(), Fraction(9, 4))
    assert (m["i"], m["j"]) == (i, j) and abs(m["r_min"] - float(v) ** 0.5) < 1e-15
    with pytest.raises(oracle.OracleError):
        oracle.min_secant(np.zeros((3, 2)), P)   # every pair a duplicate


# ---------------------------------------------------------------- update

def _setup_step(seed=1, n=12, k=4, N=60):
    w = sap_inputs.make("trig64", N=N, seed=seed)
    X = w.X.astype(np.float64)[:, :n]
    rng = np.random.default_rng(seed)
    P = sap_inputs.random_orthonormal(rng, n, k)
    m = oracle.min_secant(X, P)
    s, _ = oracle.unit_secant(X, m["i"], m["j"])
    return P, s, m


@pytest.mark.parametrize("alpha", [0.01, 0.3, 0.9])
def test_step_closed_form_new_norm(alpha):
    """P7: after one update the old worst secant has
    ||P'^T s|| = ((1-a) a_^2 + a b^2) / sqrt((1-a)^2 a_^2 + a^2 b^2),
    a_ = ||P P^T s||, b = sqrt(1 - a_^2) (the other new basis vectors are
    orthogonal to s)."""
    P, s, m = _setup_step()
    P2, _ = oracle.step(P, s, alpha)
    a = np.linalg.norm(P.T @ s); b = np.sqrt(1 - a * a)
    pred = ((1 - alpha) * a * a + alpha * b * b) / np.sqrt((1 - alpha) ** 2 * a * a + alpha ** 2 * b * b)
    assert abs(np.linalg.norm(P2.T @ s) - pred) < 1e-14
    assert oracle.orth_error(P2) < 1e-14


def test_step_principal_angles_and_projector():
    """P8: span(P') = span(P) minus v^ plus u, so the principal cosines of
    (P, P') are (1, ..., 1, cos theta) with cos theta = (1-a)||v|| / ||(1-a)v + a(s-v)||,
    and P'P'^T = PP^T - v^ v^T + u u^T."""
    alpha = 0.01
    P, s, _ = _setup_step(seed=2)
    P2, _ = oracle.step(P, s, alpha)
    v = P @ (P.T @ s)
    uu = (1 - alpha) * v + alpha * (s - v)
    cos_t = (1 - alpha) * np.linalg.norm(v) / np.linalg.norm(uu)
    sv = np.linalg.svd(P.T @ P2, compute_uv=False)
    assert np.allclose(np.sort(sv), np.sort(np.r_[np.ones(P.shape[1] - 1), cos_t]), atol=1e-13)
    vh = v / np.linalg.norm(v); u = uu / np.linalg.norm(uu)
    proj = P @ P.T - np.outer(vh, vh) + np.outer(u, u)
    assert np.abs(P2 @ P2.T - proj).max() < 1e-13
    assert np.allclose(P2[:, 0], u, atol=1e-15)


def test_step_basis_equals_library_qr():
    """MGS of {v, p_1..p_k without p_t} and a Householder QR (numpy) of the
    same ordered vectors give the same orthonormal vectors once the QR's
    column signs are fixed to make diag(R) > 0; only the first is replaced."""
    P, s, _ = _setup_step(seed=4, n=20, k=6)
    c = P.T @ s
    t = int(np.argmax(np.abs(c)))
    v = P @ c
    A = np.column_stack([v] + [P[:, q] for q in range(P.shape[1]) if q != t])
    Q, R = np.linalg.qr(A)
    Q = Q * np.sign(np.diag(R))[None, :]
    P2, t2 = oracle.step(P, s, 0.01)
    assert t2 == t
    assert np.abs(P2[:, 1:] - Q[:, 1:]).max() < 1e-13


def test_step_argmax_tie_takes_first():
    """Ties in |<p_c, s>| go to the smallest index (reading of the argmax step)."""
    P = np.eye(4)[:, :3]
    s = np.array([0.0, 1.0, -1.0, 1.0]) / np.sqrt(3.0)      # |c| = (0, a, a)
    _, t = oracle.step(P, s, 0.01)
    assert t == 1


def test_step_zero_branch():
    """P6: if every <p_c, s> is zero the paper picks p_1; the new first vector
    is s itself and P' = [s, p_2, ..., p_k]."""
    x1 = np.array([1, 0, 1, 0, 1, 0, 1, 0, 1, 0], float)
    x2 = np.array([-1, 0, 1, 0, -1, 0, 1, 0, -1, 0], float)
    X = np.stack([x1, x2])
    P = np.zeros((10, 2)); P[2, 0] = 1.0; P[3, 1] = 1.0       # [e3, e4]
    m = oracle.min_secant(X, P)
    assert m["r_min"] == 0.0
    s, d = oracle.unit_secant(X, 0, 1)
    assert d == np.sqrt(12.0)
    P2, t = oracle.step(P, s, 0.01)
    expect = np.zeros((10, 2))
    expect[[0, 4, 8], 0] = 1.0 / np.sqrt(3.0)
    expect[3, 1] = 1.0
    assert t == 0 and np.abs(P2 - expect).max() < 1e-15


@pytest.mark.parametrize("phi", [0.3, 1.2, 2.5, -0.7])
def test_step_two_points_in_plane(phi):
    """P9: N = 2, n = 2, k = 1, x_1 - x_0 = (cos phi, sin phi), P = e1.
    s = x_0 - x_1, v = (-cos phi, 0), s - v = (0, -sin phi), so
    P' = -((1-a) cos phi, a sin phi) / ||.|| (hand computation)."""
    a = 0.01
    X = np.array([[0.0, 0.0], [np.cos(phi), np.sin(phi)]])
    P = np.array([[1.0], [0.0]])
    m = oracle.min_secant(X, P)
    assert abs(m["r_min"] - abs(np.cos(phi))) < 1e-15
    s, _ = oracle.unit_secant(X, 0, 1)
    P2, _ = oracle.step(P, s, a)
    e = -np.array([(1 - a) * np.cos(phi), a * np.sin(phi)])
    e /= np.linalg.norm(e)
    assert np.abs(P2[:, 0] - e).max() < 1e-15


def test_step_rule_normalized_constant_angle():
    """Rule 1 (unit-vector reading of the shift): the rotation angle is
    atan(a / (1-a)) whatever ||v||."""
    alpha = 0.01
    for seed in (1, 5):
        P, s, _ = _setup_step(seed=seed)
        P2, _ = oracle.step(P, s, alpha, rule=1)
        sv = np.linalg.svd(P.T @ P2, compute_uv=False)
        assert abs(sv.min() - np.cos(np.arctan(alpha / (1 - alpha)))) < 1e-13


def test_orth_error_flags_non_orthonormal_bases():
    """The orthonormality checker (the max entry of |P^T P - I|) against
    values its definition fixes by hand: an off-diagonal defect with unit
    columns (a diagonal-only check would miss it), a scaled column, a column
    pair at a known angle, and exactly orthonormal bases (permuted axes, a
    rotation by a rational-cosine angle)."""
    n = 5
    e = np.eye(n)
    # unit columns at 45 degrees: P^T P = [[1, 1/sqrt2], [1/sqrt2, 1]]
    P = np.stack([e[0], (e[0] + e[1]) / np.sqrt(2.0)], axis=1)
    assert abs(oracle.orth_error(P) - 1.0 / np.sqrt(2.0)) < 1e-15
    # a column of length 2: the diagonal entry 4 - 1 = 3
    P = np.stack([2.0 * e[0], e[1], e[2]], axis=1)
    assert oracle.orth_error(P) == 3.0
    # columns (3, 4)/5 and (4, 3)/5: inner product 24/25
    P = np.zeros((n, 2))
    P[0, 0], P[1, 0], P[0, 1], P[1, 1] = 0.6, 0.8, 0.8, 0.6
    assert abs(oracle.orth_error(P) - 0.96) < 1e-15
    # a single non-unit column (k = 1): |0.5^2 - 1|
    assert oracle.orth_error(0.5 * e[:, :1]) == 0.75
    # exactly orthonormal: permuted axes, and the (3, 4, 5) rotation
    assert oracle.orth_error(e[:, [3, 0, 4]]) == 0.0
    P = np.zeros((n, 2))
    P[1, 0], P[2, 0], P[1, 1], P[2, 1] = 0.6, 0.8, -0.8, 0.6
    assert oracle.orth_error(P) <= 2.0 ** -52


# ---------------------------------------------------------------- initial projection

def test_pca_right_triangle_by_hand():
    """Algorithm 1's start, pinned by hand: the points (0,0), (1,0), (0,1)
    give the unit secants (-1,0), (0,-1), (1,-1)/sqrt2, so
    S S^T = [[3/2, -1/2], [-1/2, 3/2]]: singular values sqrt2 and 1, the
    first left singular vector (1, -1)/sqrt2."""
    X = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    S = oracle.secant_matrix(X)
    assert np.allclose(S @ S.T, [[1.5, -0.5], [-0.5, 1.5]], atol=1e-15)
    P, sv, _ = oracle.pca_init(X, 2)
    assert np.allclose(sv, [np.sqrt(2.0), 1.0], atol=1e-15)
    assert np.allclose(P[:, 0], [1 / np.sqrt(2.0), -1 / np.sqrt(2.0)], atol=1e-15)
    assert np.allclose(P[:, 1], [1 / np.sqrt(2.0), 1 / np.sqrt(2.0)], atol=1e-15)


def test_pca_regular_octagon_is_isotropic():
    """The vertices of a regular octagon: the 28 secants are invariant under
    the rotation by 45 degrees, so S S^T is a multiple of I: both singular
    values are sqrt(28 / 2)."""
    a = 2 * np.pi * np.arange(8) / 8
    X = np.stack([np.cos(a), np.sin(a)], axis=1)
    _, sv, _ = oracle.pca_init(X, 2)
    assert np.allclose(sv, [np.sqrt(14.0)] * 2, atol=1e-13)


def test_pca_planar_data_spans_the_plane():
    """Points on an affine k-plane: every secant lies in the plane, so the top
    k left singular vectors span it and the other singular values are 0."""
    rng = np.random.default_rng(5)
    A = sap_inputs.random_orthonormal(rng, 9, 3)
    X = rng.standard_normal((60, 3)) @ A.T + 0.3
    P, sv, allsv = oracle.pca_init(X, 3)
    assert np.abs(P @ P.T - A @ A.T).max() < 1e-12
    assert allsv[3:].max() < 1e-12 * allsv[0]


def test_pca_trace_counts_kept_pairs_and_is_rotation_equivariant():
    """sum sigma^2 = trace S S^T = the number of kept unit secants (with
    duplicates and a length threshold dropping some), and rotating the data
    rotates the singular vectors: P(X R^T) spans R span(P(X))."""
    w = sap_inputs.make("trig10", N=70)
    X = w.X.copy()
    X[11] = X[4]
    X[40] = X[4]
    ref = oracle.min_secant(X, w.P0, min_len=0.6)
    _, _, allsv = oracle.pca_init(X, 3, min_len=0.6)
    assert abs((allsv ** 2).sum() - ref["n_pairs"]) < 1e-9 * ref["n_pairs"]
    R = sap_inputs.random_orthonormal(np.random.default_rng(8), 10, 10)
    P, _, sv = oracle.pca_init(X, 4, min_len=0.6)
    PR, _, svR = oracle.pca_init(X @ R.T, 4, min_len=0.6)
    assert sv[3] - sv[4] > 1e-3 * sv[0]          # a gap after the fourth value
    assert np.abs(PR @ PR.T - R @ P @ P.T @ R.T).max() < 1e-10
    assert np.allclose(sv, svR, rtol=1e-12)


def test_secant_matrix_matches_the_laplacian_form():
    """S S^T by another route: sum_{i<j} w_ij (x_i - x_j)(x_i - x_j)^T with
    w_ij = 1/d_ij^2 equals X^T L X for the weighted graph Laplacian
    L = diag(W 1) - W (an identity of the weights, not the oracle's loop)."""
    w = sap_inputs.make("hyper", N=90, k=3)
    X = w.X.astype(np.float64)
    S = oracle.secant_matrix(X)
    D2 = ((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)
    Wm = np.zeros_like(D2)
    off = ~np.eye(len(X), dtype=bool)
    Wm[off] = 1.0 / D2[off]
    L = np.diag(Wm.sum(1)) - Wm
    C = X.T @ L @ X
    assert np.abs(S @ S.T - C).max() < 1e-9 * np.abs(C).max()


# ---------------------------------------------------------------- loop

def test_run_trace_and_orthonormality():
    """P12 + Algorithm 1: the loop keeps P orthonormal (<= 1e-12 after 500
    steps), the trace's entries are the evaluations of the intermediate P's,
    and two runs are identical."""
    w = sap_inputs.make("trig10", N=40)
    P, tr = oracle.run(w.X, w.P0, 500)
    assert tr["orth"].max() < 1e-12 and oracle.orth_error(P) < 1e-12
    P_b, tr_b = oracle.run(w.X, w.P0, 500)
    assert np.array_equal(P, P_b) and np.array_equal(tr["min"], tr_b["min"])
    # replay the first steps by hand through min_secant / step
    Pc = w.P0.copy()
    for it in range(4):
        m = oracle.min_secant(w.X, Pc)
        assert m["r_min"] == tr["min"][it] and (m["i"], m["j"]) == tuple(tr["ij"][it])
        s, _ = oracle.unit_secant(w.X, m["i"], m["j"])
        Pc, _ = oracle.step(Pc, s, 0.01)
    # the last entry is the evaluation of the returned P
    assert oracle.min_secant(w.X, P)["r_min"] == tr["min"][-1]


def test_run_improves_worst_secant():
    """SAP raises the minimum projected norm from a random start (Sec. 5,
    Sec. 6.2: the min generally increases with the iteration count)."""
    w = sap_inputs.make("trig10", N=100)
    _, tr = oracle.run(w.X, w.P0, 100)
    assert tr["min"][-20:].max() > 2.0 * tr["min"][0]


# ---------------------------------------------------------------- soft-min

def test_softmin_bounds_and_weights():
    """P11: r_min - tau log|Pi| <= L <= r_min, and the weights sum to 1."""
    w = sap_inputs.make("hyper", N=60)
    m = oracle.min_secant(w.X, w.P0)
    for tau in (0.01, 0.1, 1.0):
        out = oracle.softmin(w.X, w.P0, tau)
        assert m["r_min"] - tau * np.log(m["n_pairs"]) - 1e-15 <= out["L"] <= m["r_min"] + 1e-15
        assert abs(out["wsum"] - 1.0) < 1e-12
    # tau -> 0 recovers the hard min
    assert abs(oracle.softmin(w.X, w.P0, 1e-5)["L"] - m["r_min"]) < 1e-4


def test_softmin_gradient_finite_differences():
    """P11: central differences of L along random directions match <G, E>."""
    w = sap_inputs.make("trig64", N=50)
    X = w.X.astype(np.float64)
    tau = 0.05
    out = oracle.softmin(X, w.P0, tau)
    rng = np.random.default_rng(0)
    h = 1e-6
    for _ in range(3):
        E = rng.standard_normal(w.P0.shape)
        Lp = oracle.softmin(X, w.P0 + h * E, tau, grad=False)["L"]
        Lm = oracle.softmin(X, w.P0 - h * E, tau, grad=False)["L"]
        fd = (Lp - Lm) / (2 * h)
        an = float(np.sum(out["G"] * E))
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))


def test_softmin_gradient_equivariance_and_limit():
    """P11: G(PQ) = G(P) Q, G is translation invariant, and as tau -> 0 the
    gradient tends to s* (P^T s*)^T / r* of the worst secant."""
    w = sap_inputs.make("trig10", N=45)
    rng = np.random.default_rng(9)
    Q = sap_inputs.random_orthonormal(rng, w.k, w.k)
    g1 = oracle.softmin(w.X, w.P0, 0.05)["G"]
    g2 = oracle.softmin(w.X, w.P0 @ Q, 0.05)["G"]
    assert np.abs(g2 - g1 @ Q).max() < 1e-12
    g3 = oracle.softmin(w.X + 2.0, w.P0, 0.05)["G"]
    assert np.abs(g3 - g1).max() < 1e-11
    m = oracle.min_secant(w.X, w.P0)
    s, _ = oracle.unit_secant(w.X, m["i"], m["j"])
    c = w.P0.T @ s
    gap = m["r_second"] - m["r_min"]
    tau = gap / 60.0
    g0 = oracle.softmin(w.X, w.P0, tau)["G"]
    assert np.abs(g0 - np.outer(s, c) / m["r_min"]).max() < 1e-6 * np.abs(g0).max() + 1e-12


def test_softmin_zero_norm_pairs_counted():
    """A pair with r = 0 has no gradient: it adds nothing and is counted."""
    X = np.array([[0.0, 0.0], [1.0, 0.0], [0.3, 2.0]])
    P = np.array([[0.0], [1.0]])
    out = oracle.softmin(X, P, 0.1)
    assert out["n_zero"] == 1 and out["n_pairs"] == 3
