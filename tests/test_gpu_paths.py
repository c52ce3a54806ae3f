"""GPU checks of the paths a plain run rarely takes, through the C ABI:

  * the update's zero branch (Sec. 4: if every <p_c, s> is zero, p_1 is the
    vector replaced; reading: P' = [s, p_2, .., p_k]) and the normalized
    reading of the shift, each against the FP64 oracle's step;
  * candidate-list overflow: a full list keeps its smallest coarse keys and,
    when a pair of the proven window had to be dropped, the result is
    reported uncertified -- it is then still an exact FP64 value of a real
    pair, and a certified result always equals the oracle's;
  * work items whose pairs are all masked (an empty rescoring window);
  * short pairs bounded from the unrounded FP64 projection, evaluated
    exactly only where one of their block's two smallest values may lie;
  * the runner-up field against the oracle's second-smallest value;
  * the soft-min backward refusing a P other than its forward's.
"""
import numpy as np
import pytest

import oracle
import sap_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1807_03425_amd import SapContext, SapError  # noqa: E402

DEV = torch.device("cuda:0")
NEAR_TIE = 1e-6


def min_tol(r, n, k):
    return 1e-12 * r + 2.0 * np.sqrt(k) * n * 2.0 ** -53


def _ctx(X, P0, **kw):
    return SapContext(torch.from_numpy(np.ascontiguousarray(X)).to(DEV), torch.from_numpy(P0), **kw)


def _check_certified(X, P, res, tag):
    """A certified result is the oracle's (Q16 near-tie rule); its runner-up
    is exact when flagged, otherwise a lower bound."""
    ref = oracle.min_secant(X, P)
    tol = min_tol(ref["r_min"], *P.shape)
    assert res["certified"] == 1, (tag, res)
    if (res["i"], res["j"]) != (ref["i"], ref["j"]):
        assert ref["r_second"] - ref["r_min"] < NEAR_TIE, (tag, res, ref)
    assert abs(res["min_norm"] - ref["r_min"]) <= tol, (tag, res, ref)
    if res["runner_up_exact"]:
        assert abs(res["runner_up"] - ref["r_second"]) <= min_tol(ref["r_second"], *P.shape), (tag, res, ref)
    else:
        assert res["runner_up"] <= ref["r_second"] + tol, (tag, res, ref)
    return ref


def _check_valid(X, P, res, tag):
    """Any result, certified or not, is the exact FP64 value of the pair it
    names, and no smaller than the true minimum."""
    ref = oracle.min_secant(X, P)
    r_pair, _ = oracle.pair_r(X, P, res["i"], res["j"])
    tol = min_tol(ref["r_min"], *P.shape)
    assert abs(r_pair - res["min_norm"]) <= tol, (tag, res, r_pair)
    assert res["min_norm"] >= ref["r_min"] - tol, (tag, res, ref)
    if res["certified"]:
        _check_certified(X, P, res, tag)
    return ref


# ------------------------------------------------------------------ update branches

@pytest.mark.parametrize("form", ["plain", "fused"])
def test_zero_branch_through_sap_step(form):
    """Pin P6 on the device: x_1 - x_2 = (2,0,0,0,2,0,0,0,2,0) is orthogonal to
    span(P) = span(e_3, e_4), so c = P^T s = 0 exactly and the update keeps
    p_2 and replaces p_1 by s: P' = [(e_1 + e_5 + e_9)/sqrt3, e_4]."""
    X = np.array([[1, 0, 1, 0, 1, 0, 1, 0, 1, 0],
                  [-1, 0, 1, 0, -1, 0, 1, 0, -1, 0]], dtype=np.float64)
    P = np.zeros((10, 2))
    P[2, 0] = P[3, 1] = 1.0
    ctx = _ctx(X, P, form=form)
    res = ctx.step(sync=True)
    assert (res["i"], res["j"]) == (0, 1) and res["min_norm"] == 0.0 and res["t"] == 0
    P_gpu = ctx.get_P().cpu().numpy()
    expect = np.zeros((10, 2))
    expect[[0, 4, 8], 0] = 1.0 / np.sqrt(3.0)
    expect[3, 1] = 1.0
    assert np.abs(P_gpu - expect).max() < 1e-15
    s, _ = oracle.unit_secant(X, 0, 1)
    P_ref, t_ref = oracle.step(P, s, 0.01)
    assert t_ref == 0 and np.abs(P_gpu - P_ref).max() < 1e-15
    ctx.close()


@pytest.mark.parametrize("form", ["plain", "fused"])
@pytest.mark.parametrize("name,N,k", [("trig64", 300, 6), ("hyper", 260, 10)])
def test_normalized_rule_lockstep(form, name, N, k):
    """The normalized reading of the shift (unit vectors of P P^T s and
    s - P P^T s), in lockstep with the oracle's rule 1, on the register
    update (n <= 64, k <= 8) and the block-wide update."""
    w = sap_inputs.make(name, N=N, k=k)
    ctx = _ctx(w.X, w.P0, form=form, rule="normalized")
    for it in range(15):
        P = ctx.get_P().cpu().numpy()
        res = ctx.step(sync=True)
        _check_certified(w.X, P, res, f"{name}/{form}/it{it}")
        s, _ = oracle.unit_secant(w.X, res["i"], res["j"])
        P_ref, t_ref = oracle.step(P, s, w.alpha, rule=1)
        P_gpu = ctx.get_P().cpu().numpy()
        assert res["t"] == t_ref
        assert np.abs(P_gpu - P_ref).max() < 1e-12, (it, np.abs(P_gpu - P_ref).max())
    ctx.close()


# ------------------------------------------------------------------ candidate overflow

@pytest.mark.parametrize("form", ["plain", "fused"])
@pytest.mark.parametrize("cap", [0, 1, 7])
def test_overflow_all_pairs_tie_is_reported_uncertified(form, cap):
    """k = n: every pair has r = 1 up to rounding, so every pair lies in the
    proven window and every wavefront's list overflows, whatever its size.
    The result must say certified = 0, and still be the exact FP64 value of
    the pair it names (within rounding of 1)."""
    rng = np.random.default_rng(7)
    X = rng.standard_normal((300, 6))
    P = sap_inputs.random_orthonormal(rng, 6, 6)
    ctx = _ctx(X, P, form=form, cand_cap=cap)
    res = ctx.min_secant()
    assert res["certified"] == 0, res
    assert abs(res["min_norm"] - 1.0) < 1e-14
    _check_valid(X, P, res, f"tie/{form}/cap{cap}")
    ctx.close()


def _lattice():
    """Integer lattice points (a, b, c), a, b in 0..9, c in 0..4, stored in
    (a, b, c) order, padded with zeros to R^6; P = [e_1, e_2].  The pairs that
    differ only in c project to exactly 0: 1000 exact ties at r = 0, about 64
    per 32 x 64 half-tile near the diagonal."""
    a, b, c = np.meshgrid(np.arange(10), np.arange(10), np.arange(5), indexing="ij")
    X = np.zeros((500, 6))
    X[:, 0], X[:, 1], X[:, 2] = a.ravel(), b.ravel(), c.ravel()
    P = np.zeros((6, 2))
    P[0, 0] = P[1, 1] = 1.0
    return X, P


@pytest.mark.parametrize("form", ["plain", "fused"])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_zero_ties_full_list_certifies_smallest_pair(form, dtype):
    """With the full candidate list every zero-r pair of a wavefront fits:
    the result is certified and is the lexicographically smallest of the
    1000 tied pairs, (0, 1), exactly as the oracle's."""
    X, P = _lattice()
    X = X.astype(dtype)
    ctx = _ctx(X, P, form=form)
    res = ctx.min_secant()
    ref = _check_certified(X, P, res, "lattice")
    assert (res["i"], res["j"]) == (ref["i"], ref["j"]) == (0, 1) and res["min_norm"] == 0.0
    assert res["runner_up_exact"] == 1 and res["runner_up"] == 0.0
    ctx.close()


@pytest.mark.parametrize("form", ["plain", "fused"])
@pytest.mark.parametrize("cap", [1, 2, 7])
def test_zero_ties_small_list_is_reported_uncertified(form, cap):
    """The same evaluation with lists of 1, 2 or 7 entries: the wavefronts
    that hold more tied zero keys than fit must drop some, so the result is
    reported uncertified -- but still a real pair at exactly r = 0."""
    X, P = _lattice()
    ctx = _ctx(X, P, form=form, cand_cap=cap)
    res = ctx.min_secant()
    assert res["certified"] == 0, res
    assert res["min_norm"] == 0.0
    _check_valid(X, P, res, f"lattice/cap{cap}")
    ctx.close()


@pytest.mark.parametrize("form", ["plain", "fused"])
@pytest.mark.parametrize("cap", [1, 2])
def test_small_caps_never_certify_a_wrong_pair(form, cap):
    """Tiny candidate lists on a regular workload, over several starts and
    steps: every result is a real pair's exact FP64 value no smaller than the
    true minimum, and every result that claims certified = 1 is the
    oracle's."""
    w = sap_inputs.make("trig64", N=300)
    for seed in range(6):
        P = sap_inputs.random_orthonormal(np.random.default_rng(100 + seed), w.n, w.k)
        ctx = _ctx(w.X, P, form=form, cand_cap=cap)
        for it in range(4):
            Pc = ctx.get_P().cpu().numpy()
            res = ctx.step(sync=True)
            _check_valid(w.X, Pc, res, f"seed{seed}/it{it}")
        ctx.close()


@pytest.mark.parametrize("form", ["plain", "fused"])
def test_large_cap_certifies_where_small_cap_overflowed(form):
    """The same evaluations with the full list (128 per wavefront) are all
    certified and equal to the oracle's."""
    w = sap_inputs.make("trig64", N=300)
    for seed in range(6):
        P = sap_inputs.random_orthonormal(np.random.default_rng(100 + seed), w.n, w.k)
        ctx = _ctx(w.X, P, form=form)
        _check_certified(w.X, P, ctx.min_secant(), f"seed{seed}")
        ctx.close()


# ------------------------------------------------------------------ masked work items

@pytest.mark.parametrize("form", ["plain", "fused"])
def test_work_items_of_only_dropped_pairs(form):
    """Points 0..299 are one point repeated, so the first plain chunks (pairs
    (0, 1..256), ...) and the first fused tiles hold only dropped duplicate
    pairs: their smallest key is the empty marker, their window must be
    empty, and the result certified and equal to the oracle's."""
    rng = np.random.default_rng(3)
    X = rng.standard_normal((420, 8))
    X[:300] = X[0]
    P = sap_inputs.random_orthonormal(rng, 8, 3)
    ctx = _ctx(X, P, form=form)
    info = ctx.info()
    ref = _check_certified(X, P, ctx.min_secant(), f"dups/{form}")
    assert info["n_pairs"] == ref["n_pairs"] and info["n_dropped"] == ref["n_dropped"]
    assert info["n_dropped"] == 300 * 299 // 2
    ctx.close()


@pytest.mark.parametrize("form", ["plain", "fused"])
def test_work_items_of_only_short_secants(form):
    """The same with the length threshold: a tight cluster of 280 points
    whose secants are all shorter than min_len."""
    rng = np.random.default_rng(4)
    X = rng.standard_normal((400, 8))
    X[:280] = X[0] + 1e-3 * rng.standard_normal((280, 8))
    P = sap_inputs.random_orthonormal(rng, 8, 3)
    ctx = _ctx(X, P, form=form, min_len=0.05)
    ref = oracle.min_secant(X, P, min_len=0.05)
    res = ctx.min_secant()
    assert res["certified"] == 1
    assert (res["i"], res["j"]) == (ref["i"], ref["j"]) or ref["r_second"] - ref["r_min"] < NEAR_TIE
    assert abs(res["min_norm"] - ref["r_min"]) <= min_tol(ref["r_min"], 8, 3)
    assert ctx.info()["n_dropped"] == ref["n_dropped"] >= 280 * 279 // 2
    ctx.close()


# ------------------------------------------------------------------ short pairs from the FP64 Y

@pytest.mark.parametrize("name,N,k", [("trig64", 300, 6), ("blob", 260, 4), ("hyper", 330, 10)])
def test_every_pair_short_lockstep(name, N, k):
    """Every pair on the short-pair list (close_d above every distance): with
    the FP64 GEMM each pair is bounded from the unrounded Y and few are
    evaluated exactly; the results are the oracle's over a lockstep run, and
    agree with every short pair evaluated exactly (FP32 GEMM, no FP64 Y) up
    to the rounding of two FP64 evaluation orders."""
    w = sap_inputs.make(name, N=N, k=k)
    p = N * (N - 1) // 2
    kw = dict(form="fused", close_d=1e30, close_cap=p)
    a = _ctx(w.X, w.P0, gemm="f64", **kw)
    b = _ctx(w.X, w.P0, gemm="f32", **kw)
    assert a.info()["n_close"] == p
    n_exact = []
    for it in range(8):
        P = a.get_P().cpu().numpy()
        ra = a.step(sync=True)
        rb = b.step(sync=True)
        ref = _check_certified(w.X, P, ra, f"{name} it{it}")
        assert rb["certified"] == 1
        if ref["r_second"] - ref["r_min"] >= NEAR_TIE:
            assert (ra["i"], ra["j"]) == (rb["i"], rb["j"]), (it, ra, rb)
        tol = min_tol(ref["r_min"], w.n, k)
        assert abs(ra["min_norm"] - rb["min_norm"]) <= tol, (it, ra, rb)
        assert ra["runner_up_exact"] == rb["runner_up_exact"] == 1
        assert abs(ra["runner_up"] - rb["runner_up"]) <= min_tol(ref["r_second"], w.n, k)
        if (ra["i"], ra["j"]) != (rb["i"], rb["j"]):
            break                     # a near-tie resolved differently: the runs part here
        assert np.abs(a.get_P().cpu().numpy() - b.get_P().cpu().numpy()).max() < 1e-12
        n_exact.append(ra["n_rescored"])
    print(f"[short64] {name}/N{N}/k{k}: {p} short pairs, exactly evaluated per iteration "
          f"{np.mean(n_exact):.0f} (FP32 GEMM: all {p})", flush=True)
    assert max(n_exact) < p // 10
    a.close()
    b.close()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_short_pair_ties_and_runner_up(dtype):
    """The planted five-way exact tie of the runner-up test with every pair
    short: all five tied pairs are exactly evaluated, the smallest pair
    index wins and the runner-up is exact."""
    rng = np.random.default_rng(11)
    N, n, k = 300, 8, 2
    X = rng.integers(-50, 51, size=(N, n)).astype(np.float64)
    X[:, 0] = 4.0 * rng.permutation(N)
    delta = np.array([1, 0, 300, 400, 200, -100, 250, 350], dtype=np.float64)
    for a_, b_ in ((250, 260), (40, 290), (7, 8), (120, 5), (299, 150)):
        X[b_] = X[a_] + delta
    X = X.astype(dtype)
    P = np.zeros((n, k))
    P[0, 0] = P[1, 1] = 1.0
    ctx = _ctx(X, P, form="fused", close_d=1e30, close_cap=N * (N - 1) // 2)
    res = ctx.min_secant()
    ref = _check_certified(X, P, res, "short ties")
    assert (res["i"], res["j"]) == (ref["i"], ref["j"])
    assert res["runner_up_exact"] == 1 and res["runner_up"] == res["min_norm"] == ref["r_second"]
    ctx.close()


# ------------------------------------------------------------------ runner-up

@pytest.mark.parametrize("form", ["plain", "fused"])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_runner_up_of_planted_ties_is_exact(form, dtype):
    """Integer points with five translated copies of one difference vector:
    the minimum is a five-way exact tie, so the runner-up equals the minimum
    and lies inside the rescoring window (exact)."""
    rng = np.random.default_rng(11)
    N, n, k = 300, 8, 2
    X = rng.integers(-50, 51, size=(N, n)).astype(np.float64)
    X[:, 0] = 4.0 * rng.permutation(N)
    delta = np.array([1, 0, 300, 400, 200, -100, 250, 350], dtype=np.float64)
    for a, b in ((250, 260), (40, 290), (7, 8), (120, 5), (299, 150)):
        X[b] = X[a] + delta
    X = X.astype(dtype)
    P = np.zeros((n, k))
    P[0, 0] = P[1, 1] = 1.0
    ctx = _ctx(X, P, form=form)
    res = ctx.min_secant()
    ref = _check_certified(X, P, res, "ties")
    assert res["runner_up_exact"] == 1 and res["runner_up"] == res["min_norm"] == ref["r_second"]
    ctx.close()


@pytest.mark.parametrize("form", ["plain", "fused"])
def test_runner_up_bounds_on_a_run(form):
    """Over a lockstep run the runner-up is exact or a lower bound of the
    oracle's, and the gap it implies never hides a near-tie."""
    w = sap_inputs.make("trig64", N=300)
    ctx = _ctx(w.X, w.P0, form=form)
    n_exact = 0
    for it in range(25):
        P = ctx.get_P().cpu().numpy()
        res = ctx.step(sync=True)
        ref = _check_certified(w.X, P, res, f"it{it}")
        n_exact += res["runner_up_exact"]
        # a gap of at least 1e-6 by the device's bound is a true gap
        if res["runner_up"] - res["min_norm"] >= NEAR_TIE:
            assert ref["r_second"] - ref["r_min"] >= NEAR_TIE - 1e-12
    ctx.close()


# ------------------------------------------------------------------ soft-min saved state

def test_softmin_bwd_rejects_another_P():
    w = sap_inputs.make("trig64", N=200, k=6)
    ctx = _ctx(w.X, w.P0, form="fused")
    P1 = torch.from_numpy(w.P0.astype(np.float32)).to(DEV)
    P2 = P1 * 1.001
    one = torch.ones(1, device=DEV)
    ctx.softmin_fwd(P1, 0.01)
    with pytest.raises(SapError, match="INVALID_ARG"):
        ctx.softmin_bwd(P2, 0.01, one)
    g1 = ctx.softmin_bwd(P1, 0.01, one)          # the forward's P still works
    ctx.softmin_fwd(P2, 0.01)
    g2 = ctx.softmin_bwd(P2, 0.01, one)
    with pytest.raises(SapError, match="INVALID_ARG"):
        ctx.softmin_bwd(P1, 0.01, one)
    assert not torch.equal(g1, g2)
    ctx.close()


# ------------------------------------------------------------------ graph capture

def test_run_replays_from_a_captured_graph():
    """sap_run allocates, synchronises and clears nothing, so a fused run can
    be captured in a HIP graph.  An even number of iterations leaves the two
    P buffers where they started, and every replay then continues the run:
    each of three replays (with eager runs of another handle in between)
    gives the trace of the matching eager run bit for bit."""
    w = sap_inputs.make("trig64", N=300)
    iters = 4
    a = _ctx(w.X, w.P0, form="fused")
    b = _ctx(w.X, w.P0, form="fused")
    tr = dict(min=torch.empty(iters + 1, dtype=torch.float64, device=DEV),
              ij=torch.empty((iters + 1, 2), dtype=torch.int64, device=DEV),
              certified=torch.empty(iters + 1, dtype=torch.int32, device=DEV))
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        a.set_stream(s)
        with torch.cuda.graph(g, stream=s):
            a.run(iters, out=tr)
    torch.cuda.synchronize()
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        ref = b.run(iters)
        torch.cuda.synchronize()
        assert torch.equal(tr["min"], ref["min"]), rep
        assert torch.equal(tr["ij"], ref["ij"]), rep
        assert torch.equal(tr["certified"], ref["certified"]) and bool((ref["certified"] == 1).all()), rep
    assert np.array_equal(a.get_P().cpu().numpy(), b.get_P().cpu().numpy())
    a.close()
    b.close()
