"""The allocation-free batch entry point (sap_batch_run_noalloc) against the
allocating one (sap_batch_run), through the C ABI: the same kernels on the
same inputs must give the same traces and projections bit for bit, on two
calls in a row (the second smaller, so that it runs on the array the first
one left behind), and a batch above the fixed scratch fails cleanly."""
import numpy as np
import pytest

import sap_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1807_03425_amd import SapError, batch_run  # noqa: E402

DEV = torch.device("cuda:0")


def _same(a, b):
    for key in ("min", "ij", "certified"):
        assert torch.equal(a[key], b[key]), key
    for Pa, Pb in zip(a["P"], b["P"]):
        assert torch.equal(Pa, Pb)
    assert a["stats"]["n_pairs"] == b["stats"]["n_pairs"]
    assert a["stats"]["scratch_bytes"] == b["stats"]["scratch_bytes"]


def test_noalloc_matches_allocating_entry_point_twice():
    # a larger batch first: four 512-point subsamples of the hyperspectral
    # stand-in, k = 3 and 8, then a smaller one on the same array
    w = sap_inputs.make("hyper", N=3000)
    X = torch.from_numpy(w.X).to(DEV)
    sets = sap_inputs.subsample_sets(w.N, 4, 512, seed=40)
    problems = [dict(set=s, k=k) for s in range(4) for k in (3, 8)]
    P0s = sap_inputs.sweep_starts(w.n, [q["k"] for q in problems], seed=41)
    ref = batch_run(X, sets, problems, P0s, 6)
    got = batch_run(X, sets, problems, P0s, 6, noalloc=True)
    _same(ref, got)
    assert got["stats"]["init_ms"] == -1.0 and got["stats"]["run_ms"] == -1.0
    assert np.all(got["certified"].cpu().numpy() == 1)
    small_sets = [sets[1][:150], sets[3][:90]]
    small = [dict(set=0, k=2), dict(set=1, k=5)]
    P0s2 = sap_inputs.sweep_starts(w.n, [2, 5], seed=42)
    got2 = batch_run(X, small_sets, small, P0s2, 4, noalloc=True)
    ref2 = batch_run(X, small_sets, small, P0s2, 4)
    _same(ref2, got2)
    assert got2["stats"]["scratch_bytes"] < got["stats"]["scratch_bytes"]


def test_noalloc_rejects_batches_above_its_scratch():
    # 4 sets of 4096 points: 2080 tiles each, 4 x 34 MB of 1/d^2 > 32 MiB
    rng = np.random.default_rng(0)
    X = torch.from_numpy(rng.standard_normal((16384, 8))).to(DEV)
    sets = [np.arange(s * 4096, (s + 1) * 4096, dtype=np.int32) for s in range(4)]
    P0 = sap_inputs.random_orthonormal(rng, 8, 2)
    with pytest.raises(SapError, match="CAPACITY"):
        batch_run(X, sets, [dict(set=0, k=2)], [P0], 1, noalloc=True)
    # the entry point still works afterwards
    out = batch_run(X, [sets[0][:100]], [dict(set=0, k=2)], [P0], 1, noalloc=True)
    assert out["certified"][0, 0].item() == 1
