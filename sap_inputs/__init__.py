"""Seeded synthetic inputs for Secant-Avoidance Projection workloads.

This module is shared by the FP64 CPU oracle (test infrastructure) and the
HIP path.  It only *draws* inputs: point clouds X (N x n) and a starting
orthonormal projection P0 (n x k).  It holds none of the method's arithmetic
(no secants, no projected norms, no Gram-Schmidt update).

Every generator works in float64 with numpy's PCG64 and rounds once, at the
end, to the workload's storage dtype; both sides then consume those exact
bytes.  Seeds are split with ``SeedSequence(seed).spawn(2)``: child 0 draws
the data, child 1 draws P0.

Workloads (shapes follow the paper's experiments; the datasets the paper used
for its image and hyperspectral studies are not available, so synthetic
stand-ins of the same shape are drawn instead):

* ``trig``   -- trigonometric moment curve t -> (cos t, sin t, ..., cos Ht, sin Ht),
                t ~ U[0, 2pi)  (paper Sec. 5 uses H = 5, n = 10).
* ``blob``   -- 32x32 anisotropic Gaussian blob (sigma 3 px x 8 px) rotated by
                theta ~ U[0, 2pi), flattened row-major to R^1024, mean-subtracted
                (stand-in for the image data set of paper Sec. 6.2).
* ``hyper``  -- linear mixture of 5 smooth endmember spectra over 200 bands,
                Dirichlet(1) abundances, N(0, 0.01^2) noise (stand-in for the
                Indian Pines cube of paper Sec. 6.3).
* ``torus``  -- 8-torus through the (cos, sin) embedding into R^16, padded with
                N(0, 1e-3^2) noise to R^256 and rotated by a Haar orthogonal map.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

__all__ = [
    "Workload", "random_orthonormal", "trig_curve", "rotated_blob",
    "hyperspectral", "gaussian_torus", "embedded_manifold", "subsample_sets",
    "sweep_starts", "make", "WORKLOADS",
]


@dataclasses.dataclass
class Workload:
    name: str
    X: np.ndarray            # N x n, row-major, float64 or float32
    P0: np.ndarray           # n x k, float64, orthonormal columns
    k: int
    iters: int
    form: str                # "plain" | "fused" | "both"
    alpha: float = 0.01
    min_len: float = 0.0
    tau: Optional[float] = None
    note: str = ""

    @property
    def N(self) -> int:
        return int(self.X.shape[0])

    @property
    def n(self) -> int:
        return int(self.X.shape[1])

    @property
    def n_pairs(self) -> int:
        return self.N * (self.N - 1) // 2


def _rngs(seed: int):
    a, b = np.random.SeedSequence(seed).spawn(2)
    return np.random.default_rng(a), np.random.default_rng(b)


def random_orthonormal(rng: np.random.Generator, n: int, k: int) -> np.ndarray:
    """n x k with orthonormal columns: QR of an N(0,1) matrix, signs fixed so
    that diag(R) > 0 (this makes the draw Haar-distributed and reproducible)."""
    G = rng.standard_normal((n, k))
    Q, R = np.linalg.qr(G)
    sgn = np.sign(np.diag(R))
    sgn[sgn == 0] = 1.0
    return np.ascontiguousarray(Q * sgn[None, :])


def trig_curve(N: int, harmonics: int, seed: int, dtype=np.float64,
               k: int = 3, noise: float = 0.0) -> tuple[np.ndarray, np.ndarray]:
    rd, rp = _rngs(seed)
    t = rd.uniform(0.0, 2.0 * np.pi, size=N)
    h = np.arange(1, harmonics + 1, dtype=np.float64)
    ht = t[:, None] * h[None, :]
    X = np.empty((N, 2 * harmonics), dtype=np.float64)
    X[:, 0::2] = np.cos(ht)
    X[:, 1::2] = np.sin(ht)
    if noise > 0.0:
        X += rd.normal(0.0, noise, size=X.shape)
    P0 = random_orthonormal(rp, 2 * harmonics, k)
    return np.ascontiguousarray(X.astype(dtype)), P0


def rotated_blob(N: int, seed: int, k: int = 2, side: int = 32,
                 sx: float = 3.0, sy: float = 8.0) -> tuple[np.ndarray, np.ndarray]:
    rd, rp = _rngs(seed)
    theta = rd.uniform(0.0, 2.0 * np.pi, size=N)
    c0 = (side - 1) / 2.0
    rows, cols = np.meshgrid(np.arange(side, dtype=np.float64),
                             np.arange(side, dtype=np.float64), indexing="ij")
    du = (cols - c0).reshape(-1)          # horizontal offset
    dv = (rows - c0).reshape(-1)          # vertical offset
    ct, st = np.cos(theta)[:, None], np.sin(theta)[:, None]
    # coordinates in the blob's own frame: rotate the offset by -theta
    up = ct * du[None, :] + st * dv[None, :]
    vp = -st * du[None, :] + ct * dv[None, :]
    X = np.exp(-up * up / (2 * sx * sx) - vp * vp / (2 * sy * sy))
    X -= X.mean(axis=0, keepdims=True)
    P0 = random_orthonormal(rp, side * side, k)
    return np.ascontiguousarray(X.astype(np.float32)), P0


def hyperspectral(N: int, seed: int, k: int = 10, bands: int = 200,
                  endmembers: int = 5, bumps: int = 8,
                  noise: float = 0.01) -> tuple[np.ndarray, np.ndarray]:
    rd, rp = _rngs(seed)
    b = np.arange(bands, dtype=np.float64)
    E = np.zeros((endmembers, bands))
    for e in range(endmembers):
        mu = rd.uniform(0.0, bands, size=bumps)
        w = rd.uniform(4.0, 20.0, size=bumps)
        A = rd.uniform(0.1, 1.0, size=bumps)
        E[e] = (A[:, None] * np.exp(-(b[None, :] - mu[:, None]) ** 2
                                    / (2.0 * w[:, None] ** 2))).sum(axis=0)
    ab = rd.dirichlet(np.ones(endmembers), size=N)
    X = ab @ E + rd.normal(0.0, noise, size=(N, bands))
    P0 = random_orthonormal(rp, bands, k)
    return np.ascontiguousarray(X.astype(np.float32)), P0


def gaussian_torus(N: int, seed: int, k: int = 16, dim: int = 8, n: int = 256,
                   noise: float = 1e-3) -> tuple[np.ndarray, np.ndarray]:
    rd, rp = _rngs(seed)
    phi = rd.uniform(0.0, 2.0 * np.pi, size=(N, dim))
    Z = np.empty((N, n), dtype=np.float64)
    Z[:, 0:2 * dim:2] = np.cos(phi)
    Z[:, 1:2 * dim:2] = np.sin(phi)
    Z[:, 2 * dim:] = rd.normal(0.0, noise, size=(N, n - 2 * dim))
    Q = random_orthonormal(rd, n, n)       # Haar rotation of R^n
    X = Z @ Q.T
    P0 = random_orthonormal(rp, n, k)
    return np.ascontiguousarray(X.astype(np.float32)), P0


def embedded_manifold(kind: str, N: int, seed: int, n: int = 15,
                      quad: float = 0.5) -> np.ndarray:
    """Points sampled uniformly from a small manifold and smoothly embedded
    into R^n (the sweep of the paper's Sec. 6.1, whose embedding is not
    stated): base points z of
      "curve"  -- t -> (cos t, sin t, cos 2t), t ~ U[0, 2pi)        (R^3)
      "torus"  -- the torus of radii 2 and 1 in R^3, angles uniform  (R^3)
      "sphere" -- the unit 3-sphere in R^4, normalised Gaussians     (R^4)
    are mapped to [z, quad * (z_a z_b)_{a <= b}] (a smooth, non-linear
    embedding), zero-padded to R^n and rotated by a Haar orthogonal matrix.
    FP64."""
    rd = np.random.default_rng(np.random.SeedSequence(seed).spawn(2)[0])
    if kind == "curve":
        t = rd.uniform(0.0, 2.0 * np.pi, size=N)
        Z = np.stack([np.cos(t), np.sin(t), np.cos(2 * t)], axis=1)
    elif kind == "torus":
        u = rd.uniform(0.0, 2.0 * np.pi, size=N)
        v = rd.uniform(0.0, 2.0 * np.pi, size=N)
        Z = np.stack([(2.0 + np.cos(v)) * np.cos(u), (2.0 + np.cos(v)) * np.sin(u), np.sin(v)], axis=1)
    elif kind == "sphere":
        G = rd.standard_normal((N, 4))
        Z = G / np.linalg.norm(G, axis=1, keepdims=True)
    else:
        raise KeyError(kind)
    d = Z.shape[1]
    quads = [Z[:, a] * Z[:, b] for a in range(d) for b in range(a, d)]
    F = np.concatenate([Z, quad * np.stack(quads, axis=1)], axis=1)
    if F.shape[1] > n:
        raise ValueError("embedding dimension too small")
    E = np.zeros((N, n))
    E[:, :F.shape[1]] = F
    Q = random_orthonormal(rd, n, n)
    return np.ascontiguousarray(E @ Q.T)


def subsample_sets(N: int, count: int, size: int, seed: int) -> list:
    """`count` random subsets of `size` distinct rows of an N-point set (the
    sampling of the paper's Sec. 6.3), each in increasing row order."""
    rd = np.random.default_rng(seed)
    return [np.sort(rd.choice(N, size=size, replace=False)).astype(np.int32) for _ in range(count)]


def sweep_starts(n: int, ks, seed: int) -> list:
    """One seeded random orthonormal n x k start per k of a sweep."""
    rp = np.random.default_rng(seed)
    return [random_orthonormal(rp, n, int(k)) for k in ks]


def make(name: str, N: Optional[int] = None, k: Optional[int] = None,
         seed: Optional[int] = None) -> Workload:
    """Build one of the named workloads, optionally at a reduced point count
    (same recipe, fewer points) for tests that the oracle must finish fast."""
    if name == "trig10":                      # paper Sec. 5 curve, N=200
        N = N or 200; k = k or 3; seed = 1 if seed is None else seed
        X, P0 = trig_curve(N, 5, seed, np.float64, k)
        return Workload(name, X, P0, k, 200, "plain",
                        note="trig moment curve R^10, FP64")
    if name == "trig64":                      # harmonics 1..32, FP32
        N = N or 4000; k = k or 6; seed = 2 if seed is None else seed
        X, P0 = trig_curve(N, 32, seed, np.float32, k)
        return Workload(name, X, P0, k, 500, "both",
                        note="trig moment curve R^64, FP32")
    if name == "blob":
        N = N or 8000; k = k or 2; seed = 3 if seed is None else seed
        X, P0 = rotated_blob(N, seed, k)
        return Workload(name, X, P0, k, 300, "fused",
                        note="rotated 32x32 anisotropic Gaussian blob, FP32")
    if name == "hyper":
        N = N or 20000; k = k or 10; seed = 4 if seed is None else seed
        X, P0 = hyperspectral(N, seed, k)
        return Workload(name, X, P0, k, 200, "fused", tau=0.01,
                        note="synthetic hyperspectral mixture, FP32")
    if name == "torus":
        N = N or 40000; k = k or 16; seed = 5 if seed is None else seed
        X, P0 = gaussian_torus(N, seed, k)
        return Workload(name, X, P0, k, 100, "fused", tau=0.01,
                        note="8-torus rotated into R^256, FP32")
    raise KeyError(name)


WORKLOADS = ("trig10", "trig64", "blob", "hyper", "torus")
