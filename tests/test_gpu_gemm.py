"""GPU checks of the fused form with a low-precision Y = (X - mean) P GEMM
(SAP_GEMM_F32: FP32 operands, SAP_GEMM_BF16: BF16 operands; FP32
accumulation on the matrix cores), through the C ABI, against the FP64 oracle
in lockstep (the oracle evaluates the device's P at every step).

The coarse error bound widens with the operands' rounding -- the handle's
e_abs is 2 delta sqrt(w_max) with delta = R (u32 + FP64 terms) for the FP64
GEMM, sqrt(k) (n + 3) u32 R for FP32, sqrt(k) (2^-7 + 2^-15 + (n + 1) u32) R
for BF16 -- so more pairs fall in the rescoring window and the short-pair
cutoff grows.  Bars:
  * a certified result is the oracle's (argmin unless the oracle's runner-up
    is within 1e-6; min within 1e-12 relative plus 2 sqrt(k) n 2^-53);
  * an uncertified result (candidate lists that overflowed, the best of the
    rescored pairs) is a real pair's exact FP64 value within 1e-3 relative
    of the oracle's minimum;
  * the update from the reported pair equals the oracle's to 1e-12;
  * e_abs grows by the ratio of the bounds at a fixed short-pair cutoff.
The certification rate and the rescored-pair counts are printed per case.
"""
import numpy as np
import pytest

import oracle
import sap_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1807_03425_amd import SapContext  # noqa: E402

DEV = torch.device("cuda:0")
NEAR_TIE = 1e-6
U32 = 2.0 ** -24
U64 = 2.0 ** -53


def min_tol(r, n, k):
    return 1e-12 * r + 2.0 * np.sqrt(k) * n * 2.0 ** -53


def _lockstep(w, gemm, iters):
    ctx = SapContext(torch.from_numpy(w.X).to(DEV), torch.from_numpy(w.P0), form="fused",
                     alpha=w.alpha, gemm=gemm)
    info = ctx.info()
    n_cert, n_res, worst = 0, [], 0.0
    for it in range(iters):
        P = ctx.get_P().cpu().numpy()
        res = ctx.step(sync=True)
        ref = oracle.min_secant(w.X, P)
        r_pair, _ = oracle.pair_r(w.X, P, res["i"], res["j"])
        assert abs(r_pair - res["min_norm"]) <= min_tol(r_pair, w.n, w.k), (it, res, r_pair)
        if res["certified"]:
            n_cert += 1
            if (res["i"], res["j"]) != (ref["i"], ref["j"]):
                assert ref["r_second"] - ref["r_min"] < NEAR_TIE, (it, res, ref)
            assert abs(res["min_norm"] - ref["r_min"]) <= min_tol(ref["r_min"], w.n, w.k), (it, res, ref)
        else:
            rel = (res["min_norm"] - ref["r_min"]) / ref["r_min"]
            worst = max(worst, rel)
            # no smaller than the minimum (up to the two FP64 evaluations'
            # rounding) and within 1e-3 of it
            assert -min_tol(ref["r_min"], w.n, w.k) <= res["min_norm"] - ref["r_min"] <= 1e-3 * ref["r_min"], \
                (it, res, ref)
        n_res.append(res["n_rescored"])
        s, _ = oracle.unit_secant(w.X, res["i"], res["j"])
        P_ref, _ = oracle.step(P, s, w.alpha)
        assert np.abs(ctx.get_P().cpu().numpy() - P_ref).max() < 1e-12, it
    ctx.close()
    return dict(cert=n_cert / iters, rescored=float(np.mean(n_res)), e_abs=info["e_abs"],
                n_close=info["n_close"], worst_rel=worst)


@pytest.mark.parametrize("gemm", ["f32", "bf16"])
@pytest.mark.parametrize("name,N,k", [("trig64", 300, 6), ("blob", 260, 2), ("blob", 260, 8),
                                      ("hyper", 330, 10), ("torus", 200, 16)])
def test_low_precision_gemm_lockstep(gemm, name, N, k):
    w = sap_inputs.make(name, N=N, k=k)
    ref64 = _lockstep(w, "f64", 6)
    got = _lockstep(w, gemm, 6)
    print(f"[gemm] {name}/N{N}/k{k}: {gemm}: certified {got['cert']:.2f} (f64 {ref64['cert']:.2f}), "
          f"rescored/iter {got['rescored']:.0f} (f64 {ref64['rescored']:.0f}), short pairs {got['n_close']} "
          f"(f64 {ref64['n_close']}), e_abs {got['e_abs']:.2e} (f64 {ref64['e_abs']:.2e}), "
          f"worst uncertified rel err {got['worst_rel']:.1e}", flush=True)
    assert ref64["cert"] == 1.0


@pytest.mark.parametrize("name,N,k", [("trig64", 300, 6), ("hyper", 330, 10)])
def test_window_growth_matches_the_bound(name, N, k):
    """At one fixed short-pair cutoff the coarse bound's e_abs scales by
    delta(gemm) / delta(f64), the ratio the rounding analysis gives."""
    w = sap_inputs.make(name, N=N, k=k)
    X = torch.from_numpy(w.X).to(DEV)
    e = {}
    for g in ("f64", "f32", "bf16"):
        ctx = SapContext(X, torch.from_numpy(w.P0), form="fused", gemm=g, close_d=0.05,
                         close_cap=N * (N - 1) // 2)
        e[g] = ctx.info()["e_abs"]
        ctx.close()
    n, sk = w.n, np.sqrt(k)
    d64 = U32 * 1.001 + (n + 2) * sk * U64 * 4.0
    d32 = sk * (n + 3) * U32 * 1.01
    d16 = sk * (2.0 ** -7 + 2.0 ** -15 + (n + 1) * U32) * 1.01
    assert abs(e["f32"] / e["f64"] - d32 / d64) < 1e-9 * d32 / d64
    assert abs(e["bf16"] / e["f64"] - d16 / d64) < 1e-9 * d16 / d64
    print(f"[gemm] {name}: e_abs f64 {e['f64']:.2e}, f32 {e['f32']:.2e} (x{d32 / d64:.0f}), "
          f"bf16 {e['bf16']:.2e} (x{d16 / d64:.0f})", flush=True)


@pytest.mark.parametrize("gemm,L_gate,G_gate", [("f32", 1e-4, 1e-3), ("bf16", 5e-2, 5e-2)])
def test_softmin_with_low_precision_gemm(gemm, L_gate, G_gate):
    """The soft-min forward and backward from a low-precision Y: measured
    errors against the oracle, gated at 1e-4 / 1e-3 (FP32) and 5e-2 (BF16)."""
    for name, N, k in (("hyper", 400, 10), ("torus", 300, 16)):
        w = sap_inputs.make(name, N=N, k=k)
        ctx = SapContext(torch.from_numpy(w.X).to(DEV), torch.from_numpy(w.P0), form="fused", gemm=gemm)
        P32 = torch.from_numpy(w.P0.astype(np.float32)).to(DEV)
        L = float(ctx.softmin_fwd(P32, 0.01).item())
        G = ctx.softmin_bwd(P32, 0.01, torch.ones(1, device=DEV)).double().cpu().numpy()
        ctx.close()
        ref = oracle.softmin(w.X, w.P0.astype(np.float32).astype(np.float64), 0.01)
        eL = abs(L - ref["L"]) / abs(ref["L"])
        eG = np.linalg.norm(G - ref["G"]) / np.linalg.norm(ref["G"])
        print(f"[gemm] soft-min {name} {gemm}: L rel err {eL:.2e}, gradient rel err {eG:.2e}", flush=True)
        assert eL <= L_gate and eG <= G_gate, (name, gemm, eL, eG)
