"""Full-size oracle parity of every measured workload, through the C ABI.

Every check feeds the FP64 oracle the GPU's P bytes (lockstep: a trajectory
that meets a near-tie may legitimately branch) and compares the oracle's
brute-force evaluation of all N(N-1)/2 explicit unit secants with the
device's certified result:
  * argmin identical unless the oracle's runner-up lies within 1e-6 of its
    minimum (then the device's pair must score within 1e-6 of it);
  * min within 1e-12 relative plus 2 sqrt(k) n 2^-53 (both sides evaluate the
    winner in FP64 from the same input bytes);
  * the updated basis within 1e-12 of the oracle's update from the same P
    and pair.

Workloads (seeded, synthetic; sap_inputs):
  trig64  N=4000, n=64, k=6, FP32     -- all 500 iterations, fused and plain
  blob    N=8000, n=1024, k=2/4/8     -- iterations 0, 1, 2; the first step with
                                         the BF16 Y GEMM the configuration names
  hyper   N=20000, n=200, k=10        -- iterations 0, 1, 2; soft-min fwd+bwd
  torus   N=40000, n=256, k=16        -- iteration 0 (FP64 and BF16 Y GEMM);
                                         soft-min at full size (properties) and
                                         at N=4000 (oracle)
The oracle runs on the host's cores (OpenMP) and takes several minutes in all.
"""
import time

import numpy as np
import pytest

import oracle
import sap_inputs

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.fullsize]

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1807_03425_amd import SapContext  # noqa: E402

DEV = torch.device("cuda:0")
NEAR_TIE = 1e-6
BASIS_TOL = 1e-12


def min_tol(r, n, k):
    return 1e-12 * r + 2.0 * np.sqrt(k) * n * 2.0 ** -53


def _say(msg):
    print(f"[fullsize] {msg}", flush=True)


_ORACLE = {}


def _oracle_min(name, X, P):
    """oracle.min_secant, remembered per workload and P bytes (the FP64 and
    BF16 checks of one workload both evaluate its seeded start)."""
    key = (name, P.tobytes())
    if key not in _ORACLE:
        t = time.time()
        _ORACLE[key] = oracle.min_secant(X, P)
        _say(f"{name}: oracle {time.time() - t:.1f}s over {_ORACLE[key]['n_pairs']} pairs")
    return _ORACLE[key]


def _compare(Xnp, P, res, ref, tag):
    tol = min_tol(ref["r_min"], *P.shape)
    assert res["certified"] == 1, (tag, res)
    if (res["i"], res["j"]) != (ref["i"], ref["j"]):
        assert ref["r_second"] - ref["r_min"] < NEAR_TIE, (tag, res, ref)
        r_gpu_pair, _ = oracle.pair_r(Xnp, P, res["i"], res["j"])
        assert r_gpu_pair <= ref["r_min"] + NEAR_TIE, (tag, res, ref)
    assert abs(res["min_norm"] - ref["r_min"]) <= tol, (tag, res, ref)
    if res["runner_up_exact"]:
        assert abs(res["runner_up"] - ref["r_second"]) <= min_tol(ref["r_second"], *P.shape), (tag, res, ref)
    else:
        assert res["runner_up"] <= ref["r_second"] + tol, (tag, res, ref)


def _check_step(Xnp, P, res, P_gpu, alpha, tag):
    s, _ = oracle.unit_secant(Xnp, res["i"], res["j"])
    P_ref, t_ref = oracle.step(P, s, alpha)
    assert res["t"] == t_ref, (tag, res["t"], t_ref)
    err = np.abs(P_gpu - P_ref).max()
    assert err < BASIS_TOL, (tag, err)


def test_trig64_all_500_iterations_fused_and_plain():
    """The fused-vs-plain workload over its whole run: both forms step in
    lockstep with the oracle at every one of the 500 iterations.  Where the
    plain form's P equals the fused form's bit for bit (the same FP64 update
    of the same pair), the oracle's evaluation of that P is shared."""
    w = sap_inputs.make("trig64")
    X = torch.from_numpy(w.X).to(DEV)
    fused = SapContext(X, torch.from_numpy(w.P0), form="fused", alpha=w.alpha)
    plain = SapContext(X, torch.from_numpy(w.P0), form="plain", alpha=w.alpha)
    t0 = time.time()
    shared = 0
    for it in range(w.iters):
        Pf = fused.get_P().cpu().numpy()
        Pp = plain.get_P().cpu().numpy()
        rf = fused.step(sync=True)
        rp = plain.step(sync=True)
        ref = oracle.min_secant(w.X, Pf)
        _compare(w.X, Pf, rf, ref, f"fused/it{it}")
        _check_step(w.X, Pf, rf, fused.get_P().cpu().numpy(), w.alpha, f"fused/it{it}")
        if np.array_equal(Pp, Pf):
            shared += 1
            ref_p = ref
        else:
            ref_p = oracle.min_secant(w.X, Pp)
        _compare(w.X, Pp, rp, ref_p, f"plain/it{it}")
        _check_step(w.X, Pp, rp, plain.get_P().cpu().numpy(), w.alpha, f"plain/it{it}")
        if it % 100 == 0:
            _say(f"trig64 it {it}: min {rf['min_norm']:.6f} ({time.time() - t0:.0f}s)")
    _say(f"trig64: 500 iterations, plain P equal to fused P at {shared}")
    assert oracle.orth_error(fused.get_P().cpu().numpy()) < 1e-12
    fused.close()
    plain.close()


@pytest.mark.parametrize("k", [2, 4, 8])
def test_blob_iterations_0_1_2(k):
    w = sap_inputs.make("blob", k=k)
    ctx = SapContext(torch.from_numpy(w.X).to(DEV), torch.from_numpy(w.P0), form="fused", alpha=w.alpha)
    for it in range(3):
        P = ctx.get_P().cpu().numpy()
        res = ctx.step(sync=True)
        ref = _oracle_min(f"blob{k}", w.X, P)
        _say(f"blob k={k} it {it}: n_rescored {res['n_rescored']}")
        _compare(w.X, P, res, ref, f"blob{k}/it{it}")
        _check_step(w.X, P, res, ctx.get_P().cpu().numpy(), w.alpha, f"blob{k}/it{it}")
    ctx.close()


def _bf16_first_step(name, k):
    """The configuration's own arithmetic -- BF16 Y GEMM, FP32 coarse pass,
    FP64 rescoring: the first evaluation against the oracle.  Certified: the
    oracle's pair and value; otherwise (overflowing candidate lists) a real
    pair's exact value within 1e-3 of the oracle's minimum.  The update is
    checked either way."""
    w = sap_inputs.make(name, k=k)
    ctx = SapContext(torch.from_numpy(w.X).to(DEV), torch.from_numpy(w.P0), form="fused", alpha=w.alpha,
                     gemm="bf16")
    info = ctx.info()
    P = ctx.get_P().cpu().numpy()
    res = ctx.step(sync=True)
    ref = _oracle_min(f"{name}{k}", w.X, P)
    r_pair, _ = oracle.pair_r(w.X, P, res["i"], res["j"])
    assert abs(r_pair - res["min_norm"]) <= min_tol(r_pair, w.n, k)
    if res["certified"]:
        _compare(w.X, P, res, ref, f"{name}{k}/bf16")
    else:
        # no smaller than the minimum (up to the two FP64 evaluations' rounding)
        # and within 1e-3 of it
        dm = res["min_norm"] - ref["r_min"]
        assert -min_tol(ref["r_min"], w.n, k) <= dm <= 1e-3 * ref["r_min"], (res, ref)
    _check_step(w.X, P, res, ctx.get_P().cpu().numpy(), w.alpha, f"{name}{k}/bf16")
    _say(f"{name} k={k} bf16: certified {res['certified']}, rel err "
         f"{(res['min_norm'] - ref['r_min']) / ref['r_min']:.1e}, rescored {res['n_rescored']}, "
         f"short pairs {info['n_close']}, e_abs {info['e_abs']:.2e}")
    ctx.close()


@pytest.mark.parametrize("k", [2, 4, 8])
def test_blob_bf16_gemm_first_step(k):
    _bf16_first_step("blob", k)


def test_hyper_iterations_0_1_2():
    w = sap_inputs.make("hyper")
    ctx = SapContext(torch.from_numpy(w.X).to(DEV), torch.from_numpy(w.P0), form="fused", alpha=w.alpha)
    for it in range(3):
        P = ctx.get_P().cpu().numpy()
        res = ctx.step(sync=True)
        t = time.time()
        ref = oracle.min_secant(w.X, P)
        _say(f"hyper it {it}: oracle {time.time() - t:.1f}s")
        _compare(w.X, P, res, ref, f"hyper/it{it}")
        _check_step(w.X, P, res, ctx.get_P().cpu().numpy(), w.alpha, f"hyper/it{it}")
    ctx.close()


def test_torus_iteration_0():
    w = sap_inputs.make("torus")
    ctx = SapContext(torch.from_numpy(w.X).to(DEV), torch.from_numpy(w.P0), form="fused", alpha=w.alpha)
    P = ctx.get_P().cpu().numpy()
    res = ctx.step(sync=True)
    ref = _oracle_min("torus16", w.X, P)
    _compare(w.X, P, res, ref, "torus/it0")
    _check_step(w.X, P, res, ctx.get_P().cpu().numpy(), w.alpha, "torus/it0")
    ctx.close()


def test_torus_bf16_gemm_first_step():
    _bf16_first_step("torus", 16)


# ------------------------------------------------------------------ soft-min

SM_L_RTOL = 1e-5      # |dL| / |L|
SM_G_RTOL = 1e-4      # relative Frobenius error of the gradient


def _softmin_vs_oracle(w, tau, tag):
    ctx = SapContext(torch.from_numpy(w.X).to(DEV), torch.from_numpy(w.P0), form="fused")
    P32 = torch.from_numpy(w.P0.astype(np.float32)).to(DEV)
    L = float(ctx.softmin_fwd(P32, tau).item())
    G = ctx.softmin_bwd(P32, tau, torch.ones(1, device=DEV)).double().cpu().numpy()
    ctx.close()
    Pq = w.P0.astype(np.float32).astype(np.float64)
    t = time.time()
    ref = oracle.softmin(w.X, Pq, tau)
    eL = abs(L - ref["L"]) / abs(ref["L"])
    eG = np.linalg.norm(G - ref["G"]) / np.linalg.norm(ref["G"])
    _say(f"{tag}: oracle {time.time() - t:.1f}s, L {L:.8g} vs {ref['L']:.8g} (rel {eL:.2e}), "
         f"grad rel {eG:.2e}")
    assert eL <= SM_L_RTOL, (tag, L, ref["L"], eL)
    assert eG <= SM_G_RTOL, (tag, eG)


def test_softmin_hyper_full_size_against_oracle():
    """The 20,000-pixel soft-min workload (2.0e8 pairs), loss and gradient
    against the oracle's explicit-secant sums."""
    _softmin_vs_oracle(sap_inputs.make("hyper"), 0.01, "hyper soft-min")


def test_softmin_torus_4000_against_oracle():
    """The torus recipe at N = 4000 (63 x 63 tiles, many rounds of the
    backward's blocks), against the oracle."""
    _softmin_vs_oracle(sap_inputs.make("torus", N=4000), 0.01, "torus soft-min N=4000")


def test_softmin_torus_full_size_properties():
    """The torus at N = 40,000 (8.0e8 pairs, k = 16): too large for the
    oracle's soft-min, so properties that hold at any size:
      * r_min - tau log |Pi| <= L <= r_min (within the coarse bound);
      * basis equivariance dL/dP(P Q) = dL/dP(P) Q;
      * the gradient against central differences of the device's loss."""
    w = sap_inputs.make("torus")
    tau = 0.01
    ctx = SapContext(torch.from_numpy(w.X).to(DEV), torch.from_numpy(w.P0), form="fused")
    info = ctx.info()
    eb = info["e_abs"] + info["e_rel"]
    P = torch.from_numpy(w.P0.astype(np.float32)).to(DEV)
    one = torch.ones(1, device=DEV)
    L = float(ctx.softmin_fwd(P, tau).item())
    G = ctx.softmin_bwd(P, tau, one).double().cpu().numpy()
    assert np.all(np.isfinite(G)) and np.linalg.norm(G) > 0
    ctx.set_P(torch.from_numpy(P.double().cpu().numpy()))
    rmin = ctx.min_secant()["min_norm"]
    assert rmin - tau * np.log(info["n_pairs"]) - 2 * eb <= L <= rmin + 2 * eb, (L, rmin)
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((w.k, w.k)))
    PQ = torch.from_numpy((P.double().cpu().numpy() @ Q).astype(np.float32)).to(DEV)
    LQ = float(ctx.softmin_fwd(PQ, tau).item())
    GQ = ctx.softmin_bwd(PQ, tau, one).double().cpu().numpy()
    assert abs(LQ - L) <= 1e-5 * abs(L) + 4 * eb
    assert np.linalg.norm(GQ - G @ Q) <= 1e-3 * np.linalg.norm(G), np.linalg.norm(GQ - G @ Q)
    h = 1e-3
    for _ in range(2):
        E = rng.standard_normal(G.shape)
        E /= np.linalg.norm(E)
        Et = torch.from_numpy(E.astype(np.float32)).to(DEV)
        Lp = float(ctx.softmin_fwd(P + h * Et, tau).item())
        Lm = float(ctx.softmin_fwd(P - h * Et, tau).item())
        fd = (Lp - Lm) / (2 * h)
        an = float((G * E).sum())
        assert abs(fd - an) <= 2e-2 * np.linalg.norm(G) + 4 * eb / h, (fd, an)
    _say(f"torus soft-min N=40000: L {L:.6g}, |G| {np.linalg.norm(G):.4g}")
    ctx.close()
