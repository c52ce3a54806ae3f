"""GPU parity of the soft-min loss and its hand-written gradient against the
FP64 oracle, through the C ABI (fused form).

Bars: |L~ - L| / |L| <= 1e-5 and a relative Frobenius error of the gradient
<= 1e-4 (FP32 coarse evaluation), each measured error printed per case.  Both
are also held to the coarse pass's proven bound |r~ - r| <= e_abs + e_rel r
(sap_info; short pairs are exact FP64): L is a smooth minimum, so
|L~ - L| <= max |r~ - r|, plus FP32 rounding of the exponentials and sums
(about 1e-5 tau) and of the stored loss (2^-24 |L|); each gradient term
w s c^T / r carries a relative error of at most about (e_abs + e_rel)/tau
(through w) + (e_abs + e_rel)/r_min (through 1/r and y_i - y_j).
"""
import numpy as np
import pytest

import oracle
import sap_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1807_03425_amd import SapContext, SapError, SoftMinSecant  # noqa: E402

DEV = torch.device("cuda:0")
L_RTOL = 1e-5
G_RTOL = 1e-4


def _ctx(X, P0, **kw):
    Xt = torch.from_numpy(X).to(DEV)
    return SapContext(Xt, torch.from_numpy(P0), form="fused", **kw), Xt


def _tols(info, tau, L, rmin, pnorm=1.0):
    # the coarse bound is stated for ||P||_2 <= 1; it scales with ||P||_2
    eb = (info["e_abs"] + info["e_rel"]) * max(pnorm, 1.0)
    tol_L = 2.0 * eb + 1e-5 * tau + 2.0 ** -23 * abs(L)
    tol_G = 4.0 * (eb / tau + eb / max(rmin, 1e-3)) + 1e-5
    return tol_L, tol_G


def _compare(X, P, tau, tag, min_len=0.0, P_init=None, **kw):
    # the handle is created with an orthonormal P (sap_init checks it); the
    # soft-min takes any P
    ctx, _ = _ctx(X, P if P_init is None else P_init, min_len=min_len, **kw)
    P32 = torch.from_numpy(P.astype(np.float32)).to(DEV)
    loss = ctx.softmin_fwd(P32, tau)
    dP = ctx.softmin_bwd(P32, tau, torch.ones(1, device=DEV))
    torch.cuda.synchronize()
    Pq = P.astype(np.float32).astype(np.float64)   # the projection the GPU used
    ref = oracle.softmin(X, Pq, tau, min_len=min_len)
    rmin = oracle.min_secant(X, Pq, min_len=min_len)["r_min"]
    tol_L, tol_G = _tols(ctx.info(), tau, ref["L"], rmin, np.linalg.norm(Pq, 2))
    L = float(loss.item())
    G = dP.double().cpu().numpy()
    eL = abs(L - ref["L"]) / abs(ref["L"])
    rel = np.linalg.norm(G - ref["G"]) / np.linalg.norm(ref["G"])
    print(f"[softmin] {tag}: L {L:.8g} vs {ref['L']:.8g}: rel err {eL:.2e}; gradient rel err {rel:.2e}",
          flush=True)
    assert abs(L - ref["L"]) <= tol_L, (tag, L, ref["L"], tol_L)
    assert rel <= tol_G, (tag, rel, tol_G)
    assert eL <= L_RTOL, (tag, L, ref["L"], eL)
    assert rel <= G_RTOL, (tag, rel)
    ctx.close()
    return L, G, ref


@pytest.mark.parametrize("name,N,k,tau", [("trig64", 300, 6, 0.01), ("hyper", 500, 10, 0.01),
                                          ("torus", 400, 16, 0.01), ("blob", 300, 4, 0.02),
                                          ("trig10", 200, 3, 0.05)])
def test_softmin_matches_oracle(name, N, k, tau):
    w = sap_inputs.make(name, N=N, k=k)
    _compare(w.X, w.P0, tau, f"{name}/N{N}/k{k}")


@pytest.mark.parametrize("k", list(range(1, 17)))
def test_softmin_every_k(k):
    """Every compiled projection width K = 1..16 (each its own kernel
    instance, with its own LDS row length and matrix-core padding) on a
    multi-tile torus sample."""
    w = sap_inputs.make("torus", N=200, k=k)
    _compare(w.X, w.P0, 0.01, f"torus/N200/k{k}")


@pytest.mark.parametrize("N", [1, 63, 64, 65, 130])
def test_softmin_ragged_sizes(N):
    """One point short of, at, and past a 64-point tile; N = 1 + 1 pair."""
    w = sap_inputs.make("trig64", N=max(N, 2), k=6)
    _compare(w.X, w.P0, 0.01, f"ragged{N}")


def test_softmin_all_close_and_no_close_list():
    """The same problem with every pair on the FP64 short-pair list, and with
    no short-pair list at all: both agree with the oracle."""
    w = sap_inputs.make("trig64", N=200, k=6)
    X = w.X
    d = np.sqrt(((X[:, None, :].astype(np.float64) - X[None, :, :]) ** 2).sum(-1))
    _compare(X, w.P0, 0.01, "all-close", close_d=float(d.max()) * 2, close_cap=200 * 199 // 2)
    _compare(X, w.P0, 0.01, "no-close", close_d=0.0)


def test_softmin_masks_duplicates_and_short_secants():
    w = sap_inputs.make("trig64", N=150, k=6)
    X = w.X.copy()
    X[10] = X[3]
    X[77] = X[3]
    X[120] = X[119]
    d = np.sqrt(((X[:, None, :].astype(np.float64) - X[None, :, :]) ** 2).sum(-1))
    ell = float(np.quantile(d[np.triu_indices(len(X), 1)], 0.05))
    _compare(X, w.P0, 0.01, "dups")
    _compare(X, w.P0, 0.01, "min_len", min_len=ell)


def test_softmin_non_orthonormal_P():
    """The loss is defined for any P; here a scaled and sheared one."""
    w = sap_inputs.make("hyper", N=300, k=10)
    rng = np.random.default_rng(5)
    P = w.P0 @ (np.eye(10) + 0.1 * rng.standard_normal((10, 10))) * 1.3
    _compare(w.X, P, 0.02, "nonorth", P_init=w.P0)


def test_autograd_function():
    w = sap_inputs.make("hyper", N=300, k=10)
    ctx, _ = _ctx(w.X, w.P0)
    P = torch.from_numpy(w.P0.astype(np.float32)).to(DEV).requires_grad_(True)
    L = SoftMinSecant.apply(P, ctx, 0.01)
    (2.5 * L).backward()
    ref = ctx.softmin_bwd(P.detach(), 0.01, torch.full((1,), 2.5, device=DEV))
    assert torch.equal(P.grad, ref)
    ctx.softmin_fwd(P.detach(), 0.01)
    ref1 = ctx.softmin_bwd(P.detach(), 0.01, torch.ones(1, device=DEV))
    assert torch.allclose(ref1 * 2.5, ref, rtol=1e-6, atol=0)
    # forward A, forward B, backward A: A's saved state is recomputed first
    Pa = P.detach().clone().requires_grad_(True)
    Pb = (P.detach() * 1.01).requires_grad_(True)
    La = SoftMinSecant.apply(Pa, ctx, 0.01)
    Lb = SoftMinSecant.apply(Pb, ctx, 0.01)
    La.backward()
    assert torch.equal(Pa.grad, ref1)
    Lb.backward()
    ctx.softmin_fwd(Pb.detach(), 0.01)
    assert torch.equal(Pb.grad, ctx.softmin_bwd(Pb.detach(), 0.01, torch.ones(1, device=DEV)))
    assert not torch.equal(Pa.grad, Pb.grad)
    ctx.close()


def test_softmin_deterministic():
    w = sap_inputs.make("trig64", N=400, k=6)
    ctx, _ = _ctx(w.X, w.P0)
    P = torch.from_numpy(w.P0.astype(np.float32)).to(DEV)
    one = torch.ones(1, device=DEV)
    outs = []
    for _ in range(3):
        L = ctx.softmin_fwd(P, 0.01).clone()
        outs.append((L, ctx.softmin_bwd(P, 0.01, one)))
    for L, G in outs[1:]:
        assert torch.equal(L, outs[0][0]) and torch.equal(G, outs[0][1])
    ctx.close()


def test_softmin_errors():
    w = sap_inputs.make("trig64", N=100, k=6)
    X = torch.from_numpy(w.X).to(DEV)
    P = torch.from_numpy(w.P0.astype(np.float32)).to(DEV)
    one = torch.ones(1, device=DEV)
    plain = SapContext(X, torch.from_numpy(w.P0), form="plain")
    with pytest.raises(SapError, match="UNSUPPORTED"):
        plain.softmin_fwd(P, 0.01)
    plain.close()
    ctx = SapContext(X, torch.from_numpy(w.P0), form="fused")
    with pytest.raises(SapError, match="INVALID_ARG"):
        ctx.softmin_bwd(P, 0.01, one)          # no forward yet
    for bad in (0.0, -1.0, 1e-9, float("nan")):
        with pytest.raises(SapError, match="INVALID_ARG"):
            ctx.softmin_fwd(P, bad)
    ctx.softmin_fwd(P, 0.01)
    with pytest.raises(SapError, match="INVALID_ARG"):
        ctx.softmin_bwd(P, 0.02, one)          # tau differs from the forward
    ctx.softmin_bwd(P, 0.01, one)
    # the iteration still works on the same handle afterwards
    assert ctx.min_secant()["certified"] == 1
    ctx.close()


# ------------------------------------------------------------------ full size

def test_hyper_full_size_properties():
    """The 20,000-pixel, 200-band, k = 10 soft-min workload (2e8 pairs): too
    large for the oracle, so properties that hold at any size are checked:
      * min r - tau log |Pi| - eps <= L <= min r + eps (eps: the coarse bound);
      * basis equivariance dL/dP(P Q) = dL/dP(P) Q for orthogonal Q;
      * the gradient matches central differences of the GPU loss along
        random directions."""
    w = sap_inputs.make("hyper")
    tau = 0.01
    ctx, _ = _ctx(w.X, w.P0)
    info = ctx.info()
    eb = info["e_abs"] + info["e_rel"]
    P = torch.from_numpy(w.P0.astype(np.float32)).to(DEV)
    one = torch.ones(1, device=DEV)
    L = float(ctx.softmin_fwd(P, tau).item())
    G = ctx.softmin_bwd(P, tau, one).double().cpu().numpy()
    ctx.set_P(torch.from_numpy(P.double().cpu().numpy()))
    # the FP32 P is orthonormal to ~1e-7: set_P accepts it, min_secant scores it
    rmin = ctx.min_secant()["min_norm"]
    assert rmin - tau * np.log(info["n_pairs"]) - 2 * eb <= L <= rmin + 2 * eb, (L, rmin)
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((w.k, w.k)))
    PQ = torch.from_numpy((P.double().cpu().numpy() @ Q).astype(np.float32)).to(DEV)
    LQ = float(ctx.softmin_fwd(PQ, tau).item())
    GQ = ctx.softmin_bwd(PQ, tau, one).double().cpu().numpy()
    assert abs(LQ - L) <= 4 * eb + 1e-6
    tol_G = 8.0 * (eb / tau + eb / rmin) + 1e-5
    assert np.linalg.norm(GQ - G @ Q) <= tol_G * np.linalg.norm(G), np.linalg.norm(GQ - G @ Q)
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
    ctx.close()
