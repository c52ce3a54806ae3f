"""GPU parity of Algorithm 1's initial projection (sap_pca_init) against the
oracle's explicit secant matrix and its library SVD (Sec. 4; Algorithm 1,
step 2), through the C ABI.

Bars: the span of the device's k vectors equals the oracle's --
max |P_g P_g^T - P_o P_o^T| <= 1e-10 -- on data whose k-th and (k+1)-th
singular values are apart (the span is then well defined; the gap is
asserted first), the k singular values within 1e-11 relative, and every
column individually (same sign convention) within 1e-9 where the
neighbouring values are apart too.
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


def _compare(X, k, tag, form="fused", min_len=0.0):
    P0 = sap_inputs.random_orthonormal(np.random.default_rng(1), X.shape[1], k)
    ctx = SapContext(torch.from_numpy(X).to(DEV), torch.from_numpy(P0), form=form, min_len=min_len)
    Pg, info = ctx.pca_init()
    Pg = Pg.cpu().numpy()
    Po, svo, allsv = oracle.pca_init(X, k, min_len=min_len)
    gap = (allsv[k - 1] - allsv[k]) / allsv[0] if k < len(allsv) else 1.0
    assert gap > 1e-3, (tag, "no gap after the k-th singular value", allsv[:k + 2])
    assert info["converged"] == 1, (tag, info)
    span = np.abs(Pg @ Pg.T - Po @ Po.T).max()
    sv_err = np.max(np.abs(np.array(info["sigma"]) - svo) / svo)
    print(f"[pca] {tag}: span err {span:.2e}, sigma rel err {sv_err:.2e}, iters {info['iters']}, "
          f"residual {info['residual']:.1e}, {info['ms']:.2f} ms", flush=True)
    assert span <= 1e-10, (tag, span)
    assert sv_err <= 1e-11, (tag, info["sigma"], svo)
    for c in range(k):
        lo = allsv[c - 1] - allsv[c] if c > 0 else np.inf
        hi = allsv[c] - allsv[c + 1] if c + 1 < len(allsv) else np.inf
        if min(lo, hi) > 1e-3 * allsv[0]:
            assert np.abs(Pg[:, c] - Po[:, c]).max() <= 1e-9, (tag, c)
    ctx.close()
    return Pg, info


@pytest.mark.parametrize("name,N,k", [("trig10", 200, 4), ("trig64", 300, 2), ("hyper", 400, 3),
                                      ("blob", 260, 2), ("torus", 300, 4)])
def test_pca_matches_explicit_svd(name, N, k):
    w = sap_inputs.make(name, N=N, k=k)
    _compare(w.X, k, f"{name}/N{N}/k{k}")


@pytest.mark.parametrize("kind,k", [("curve", 3), ("torus", 5), ("sphere", 4)])
def test_pca_manifolds_in_r15(kind, k):
    X = sap_inputs.embedded_manifold(kind, 256, 12)
    _compare(X, k, f"{kind}/k{k}", form="plain")


def test_pca_drops_duplicates_and_short_secants():
    w = sap_inputs.make("hyper", N=300, k=3)
    X = w.X.copy()
    X[7] = X[2]
    X[150] = X[2]
    _compare(X, 3, "dups+min_len", min_len=0.08)


def test_pca_sets_the_start_of_algorithm_1():
    """With set_P the result becomes the handle's P: the run starts from it,
    and its first evaluation is the oracle's evaluation of that P."""
    w = sap_inputs.make("trig64", N=300, k=6)
    ctx = SapContext(torch.from_numpy(w.X).to(DEV), torch.from_numpy(w.P0), form="fused")
    Pg, info = ctx.pca_init(set_P=True)
    assert torch.equal(ctx.get_P(), Pg)
    P = Pg.cpu().numpy()
    assert oracle.orth_error(P) < 1e-13
    res = ctx.min_secant()
    ref = oracle.min_secant(w.X, P)
    assert res["certified"] == 1 and (res["i"], res["j"]) == (ref["i"], ref["j"])
    assert abs(res["min_norm"] - ref["r_min"]) <= 1e-12 * ref["r_min"] + 2 * np.sqrt(6) * 64 * 2.0 ** -53
    ctx.close()
