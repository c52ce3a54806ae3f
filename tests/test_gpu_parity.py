"""GPU parity of the HIP path against the FP64 CPU oracle, through the C ABI.

Bars (single-evaluation and single-step parity, compared in lockstep: the
oracle is fed the GPU's P at every checked iteration, because a trajectory
that meets a near-tie may legitimately branch):
  * argmin pair identical unless the oracle's runner-up is within 1e-6 of its
    minimum; then the GPU pair must score within 1e-6 of the minimum;
  * min norm within 1e-12 relative plus 2 sqrt(k) n 2^-53 absolute: both
    sides evaluate the winning pair in FP64 from the same input bytes (the
    GPU's FP32 coarse pass only selects which pairs to rescore, inside a
    proven error window), and each FP64 dot product P^T s of a unit secant
    carries an absolute error of at most about n 2^-53 per component;
  * updated basis within 1e-12 of the oracle's update from the same P and
    pair (max abs elementwise).
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
MIN_RTOL = 1e-12
BASIS_TOL = 1e-12
NEAR_TIE = 1e-6


def _ctx(w, form, **kw):
    X = torch.from_numpy(w.X).to(DEV)
    return SapContext(X, torch.from_numpy(w.P0), form=form, alpha=w.alpha, **kw), X


def min_tol(r, n, k):
    return MIN_RTOL * r + 2.0 * np.sqrt(k) * n * 2.0 ** -53


def _check_eval(Xnp, P, res, tag=""):
    ref = oracle.min_secant(Xnp, P)
    tol = min_tol(ref["r_min"], *P.shape)
    assert res["certified"] == 1, (tag, res)
    gap = ref["r_second"] - ref["r_min"]
    if (res["i"], res["j"]) != (ref["i"], ref["j"]):
        assert gap < NEAR_TIE, (tag, res, ref)
        r_gpu_pair, _ = oracle.pair_r(Xnp, P, res["i"], res["j"])
        assert r_gpu_pair <= ref["r_min"] + NEAR_TIE, (tag, res, ref)
    assert abs(res["min_norm"] - ref["r_min"]) <= tol, (tag, res, ref)
    # the runner-up: exact when flagged, else a lower bound of the oracle's
    if res["runner_up_exact"]:
        assert abs(res["runner_up"] - ref["r_second"]) <= min_tol(ref["r_second"], *P.shape), (tag, res, ref)
    else:
        assert res["runner_up"] <= ref["r_second"] + tol, (tag, res, ref)
    return ref


def _lockstep(w, form, iters, check_every=1, **kw):
    ctx, X = _ctx(w, form, **kw)
    Xnp = w.X
    for it in range(iters):
        P = ctx.get_P().cpu().numpy()
        res = ctx.step(sync=True)
        if it % check_every == 0 or it == iters - 1:
            _check_eval(Xnp, P, res, f"{w.name}/{form}/it{it}")
            s, _ = oracle.unit_secant(Xnp, res["i"], res["j"])
            P_ref, t_ref = oracle.step(P, s, w.alpha)
            P_gpu = ctx.get_P().cpu().numpy()
            assert res["t"] == t_ref, (it, res["t"], t_ref)
            assert np.abs(P_gpu - P_ref).max() < BASIS_TOL, (it, np.abs(P_gpu - P_ref).max())
    Pf = ctx.get_P().cpu().numpy()
    assert oracle.orth_error(Pf) < 1e-12
    ctx.close()


# ------------------------------------------------------------------ small, full lockstep

def test_trig10_plain_fp64_full_run_lockstep():
    """The paper's Sec. 5 curve (N=200, R^10 -> R^3, FP64), 200 iterations."""
    _lockstep(sap_inputs.make("trig10"), "plain", 200)


@pytest.mark.parametrize("form", ["plain", "fused"])
def test_trig64_small_lockstep(form):
    """Harmonics 1..32 curve at N=300 (5 tiles of 64 + a ragged tail)."""
    _lockstep(sap_inputs.make("trig64", N=300), form, 60)


@pytest.mark.parametrize("k", [2, 4, 8])
def test_blob_small_fused_lockstep(k):
    _lockstep(sap_inputs.make("blob", N=260, k=k), "fused", 12)


def test_hyper_small_fused_lockstep():
    _lockstep(sap_inputs.make("hyper", N=330), "fused", 12)


def test_torus_small_fused_lockstep():
    _lockstep(sap_inputs.make("torus", N=200), "fused", 8)


def test_trig10_fused_fp64_data():
    _lockstep(sap_inputs.make("trig10", N=150), "fused", 30)


# ------------------------------------------------------------------ traces and determinism

@pytest.mark.parametrize("form", ["plain", "fused"])
def test_run_trace_matches_oracle_until_first_near_tie(form):
    w = sap_inputs.make("trig10", N=120)
    iters = 80
    ctx, X = _ctx(w, form)
    tr = ctx.run(iters)
    torch.cuda.synchronize()
    P_gpu = ctx.get_P().cpu().numpy()
    P_or, ot = oracle.run(w.X, w.P0, iters)
    gmin = tr["min"].cpu().numpy()
    gij = tr["ij"].cpu().numpy()
    assert np.all(tr["certified"].cpu().numpy() == 1)
    for it in range(iters + 1):
        if ot["second"][it] - ot["min"][it] < NEAR_TIE:
            break
        assert tuple(gij[it]) == tuple(ot["ij"][it]), it
        assert abs(gmin[it] - ot["min"][it]) <= 1e-10 * ot["min"][it], it
    else:
        assert np.abs(P_gpu - P_or).max() < 1e-9
    # a second run from the same start reproduces the trace bit for bit
    ctx2, _ = _ctx(w, form)
    tr2 = ctx2.run(iters)
    torch.cuda.synchronize()
    assert torch.equal(tr2["min"], tr["min"]) and torch.equal(tr2["ij"], tr["ij"])
    ctx.close(); ctx2.close()


def test_set_get_P_roundtrip_and_resume():
    w = sap_inputs.make("trig64", N=200)
    ctx, X = _ctx(w, "fused")
    ctx.run(5)
    P5 = ctx.get_P()
    tr_a = ctx.run(7)
    ctx.set_P(P5)
    tr_b = ctx.run(7)
    torch.cuda.synchronize()
    assert torch.equal(tr_a["min"], tr_b["min"]) and torch.equal(tr_a["ij"], tr_b["ij"])
    ctx.close()


@pytest.mark.parametrize("name,N,k", [("trig64", 300, 6), ("hyper", 300, 10), ("blob", 200, 8),
                                      ("hyper", 20000, 10)])
def test_fused_run_equals_steps(name, N, k):
    """sap_run in the fused form fuses each iteration's selection and update
    with the next iteration's Y GEMM (two P buffers).  It must give exactly
    what separate sap_step calls and a final sap_min_secant give: the same
    trace and the same final basis, bit for bit.  The cases cover the
    register update (n <= 64, k <= 8), the block-wide LDS update, the Y GEMM
    split over two wavefronts per tile (blob, n = 1024) and two 64-row groups
    per fused block (hyper at N = 20000: more row groups than compute
    units)."""
    w = sap_inputs.make(name, N=N, k=k)
    iters = 6
    ctx_r, _ = _ctx(w, "fused")
    tr = ctx_r.run(iters)
    torch.cuda.synchronize()
    P_run = ctx_r.get_P().cpu().numpy()
    ctx_s, _ = _ctx(w, "fused")
    steps = [ctx_s.step(sync=True) for _ in range(iters)]
    steps.append(ctx_s.min_secant())
    P_step = ctx_s.get_P().cpu().numpy()
    gmin = tr["min"].cpu().numpy()
    gij = tr["ij"].cpu().numpy()
    for it, r in enumerate(steps):
        assert (int(gij[it][0]), int(gij[it][1])) == (r["i"], r["j"]), (it, gij[it], r)
        assert gmin[it] == r["min_norm"], (it, gmin[it], r["min_norm"])
    assert np.array_equal(P_run, P_step)
    # the run resumes from its final basis: a second run continues the trajectory
    tr2 = ctx_r.run(2)
    torch.cuda.synchronize()
    ctx_s.step(sync=True)
    ctx_s.step(sync=True)
    assert np.array_equal(ctx_r.get_P().cpu().numpy(), ctx_s.get_P().cpu().numpy())
    assert float(tr2["min"][0].item()) == gmin[iters]
    ctx_r.close(); ctx_s.close()


# ------------------------------------------------------------------ edge cases

def test_two_points():
    X = np.array([[0.0, 0.0], [0.6, 0.8]])
    P = np.array([[1.0], [0.0]])
    for form in ("plain", "fused"):
        ctx = SapContext(torch.from_numpy(X).to(DEV), torch.from_numpy(P), form=form)
        res = ctx.min_secant()
        assert (res["i"], res["j"]) == (0, 1) and abs(res["min_norm"] - 0.6) < 1e-15
        ctx.close()


@pytest.mark.parametrize("N", [65, 127, 129])
@pytest.mark.parametrize("form", ["plain", "fused"])
def test_ragged_tails(N, form):
    w = sap_inputs.make("trig64", N=N)
    ctx, X = _ctx(w, form)
    _check_eval(w.X, w.P0, ctx.min_secant(), f"N={N}")
    ctx.close()


@pytest.mark.parametrize("form", ["plain", "fused"])
def test_duplicates_and_length_threshold(form):
    w = sap_inputs.make("trig10", N=90)
    X = w.X.copy()
    X[10] = X[3]
    X[50] = X[3]
    X[77] = X[20]
    for ml in (0.0, 0.7):
        ctx = SapContext(torch.from_numpy(X).to(DEV), torch.from_numpy(w.P0), form=form, min_len=ml)
        res = ctx.min_secant()
        ref = oracle.min_secant(X, w.P0, min_len=ml)
        info = ctx.info()
        assert info["n_pairs"] == ref["n_pairs"] and info["n_dropped"] == ref["n_dropped"]
        assert (res["i"], res["j"]) == (ref["i"], ref["j"])
        assert abs(res["min_norm"] - ref["r_min"]) <= min_tol(ref["r_min"], *w.P0.shape)
        ctx.close()


def test_k_equals_n_and_k_one():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((70, 5))
    for k in (5, 1):
        P = sap_inputs.random_orthonormal(rng, 5, k)
        for form in ("plain", "fused"):
            ctx = SapContext(torch.from_numpy(X).to(DEV), torch.from_numpy(P), form=form)
            res = ctx.min_secant()
            if k == 5:
                assert abs(res["min_norm"] - 1.0) < 1e-13
            else:
                _check_eval(X, P, res, f"k=1/{form}")
            ctx.close()


def test_affine_plane_min_is_one():
    rng = np.random.default_rng(11)
    A = sap_inputs.random_orthonormal(rng, 12, 3)
    X = (rng.standard_normal((150, 3)) @ A.T + 0.5).astype(np.float32)
    for form in ("plain", "fused"):
        ctx = SapContext(torch.from_numpy(X).to(DEV), torch.from_numpy(A), form=form)
        res = ctx.min_secant()
        ref = oracle.min_secant(X, A)
        assert abs(res["min_norm"] - ref["r_min"]) <= min_tol(1.0, *A.shape)
        assert abs(res["min_norm"] - 1.0) < 1e-6
        ctx.close()


def test_errors_reported():
    w = sap_inputs.make("trig10", N=50)
    X = torch.from_numpy(w.X).to(DEV)
    with pytest.raises(SapError) as e:
        SapContext(torch.zeros((5, 4), dtype=torch.float64, device=DEV),
                   torch.from_numpy(np.eye(4)[:, :2]))
    assert e.value.status == 3                       # no pairs
    Xbad = X.clone(); Xbad[7, 2] = float("nan")
    with pytest.raises(SapError) as e:
        SapContext(Xbad, torch.from_numpy(w.P0))
    assert e.value.status == 2                       # nonfinite
    with pytest.raises(SapError) as e:
        SapContext(X, torch.from_numpy(w.P0 * 1.01))
    assert e.value.status == 6                       # not orthonormal
    ctx = SapContext(X, torch.from_numpy(w.P0))
    with pytest.raises(SapError):
        ctx.set_P(torch.from_numpy(w.P0 * 2.0))
    assert ctx.min_secant()["certified"] == 1        # the handle stays usable
    ctx.close()


# ------------------------------------------------------------------ ties

@pytest.mark.parametrize("form", ["plain", "fused"])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_exact_ties_take_smallest_pair(form, dtype):
    """Integer coordinates (exact in both dtypes) and P = the first two axes;
    five translated copies of one short difference vector give pairs whose
    FP64 r are bit-identical.  The minimum is that tie, and the reported pair
    must be its lexicographically smallest (i, j), exactly as the oracle's."""
    rng = np.random.default_rng(11)
    N, n, k = 300, 8, 2
    X = rng.integers(-50, 51, size=(N, n)).astype(np.float64)
    # coordinate 0: distinct multiples of 4, so every other pair has
    # |dx_0| >= 3 and a much shorter length than delta
    X[:, 0] = 4.0 * rng.permutation(N)
    delta = np.array([1, 0, 300, 400, 200, -100, 250, 350], dtype=np.float64)
    for a, b in ((250, 260), (40, 290), (7, 8), (120, 5), (299, 150)):
        X[b] = X[a] + delta
    X = X.astype(dtype)
    P0 = np.zeros((n, k))
    P0[0, 0] = P0[1, 1] = 1.0
    ref = oracle.min_secant(X, P0)
    assert ref["r_second"] == ref["r_min"], "the planted tie is not the minimum"
    ctx = SapContext(torch.from_numpy(X).to(DEV), torch.from_numpy(P0), form=form)
    res = ctx.min_secant()
    assert res["certified"] == 1
    assert (res["i"], res["j"]) == (ref["i"], ref["j"]), (res, ref)
    assert abs(res["min_norm"] - ref["r_min"]) <= min_tol(ref["r_min"], n, k)
    ctx.close()
