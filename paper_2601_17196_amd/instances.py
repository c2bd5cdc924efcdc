"""Seeded synthetic POT workloads.

This module only draws inputs: point clouds, marginals r and c, the mass s and
the squared-Euclidean cost built from the points.  It holds none of the
solver's arithmetic, so both the HIP path and the FP64 oracle can be fed from
it.

Problem statement (Section 2.1 of the paper): C in R_+^{n x m}, r in R_+^n,
c in R_+^m and a budget s <= min(|r|_1, |c|_1).  The paper's own data (images,
point clouds, two moons) is not available, so every workload here is drawn
from a stated distribution; the shapes follow the paper's settings of a
squared-Euclidean cost normalised to max 1 (Section 4.1 and the synthetic
scalability experiment in the appendix).

Every instance is drawn from ``numpy.random.Generator(PCG64(SeedSequence([cfg, k])))``
with ``cfg`` the workload number and ``k`` the instance index.  Points are
drawn in FP64 and stored as FP32; the cost is computed in FP64 from the FP32
points, divided by its maximum and then stored as FP32 (or BF16 by
round-to-nearest-even).  Masses are FP64.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Instance",
    "sqeuclid_cost",
    "to_bf16_bits",
    "bf16_bits_to_f64",
    "uniform_pair",
    "c1",
    "c2",
    "c3",
    "c4_batch",
    "c5",
    "c5_batch",
    "small_instance",
    "WORKLOADS",
]


@dataclasses.dataclass
class Instance:
    """One POT instance.

    x, y      : FP32 points, shapes (n, d) and (m, d)
    r, c      : FP64 marginals
    s         : FP64 transported mass
    cost_scale: 1 / max_ij |x_i - y_j|^2 computed in FP64
    C64       : FP64 cost cost_scale*|x_i - y_j|^2 (the points-defined cost)
    C32       : C64 rounded to FP32 (the stored cost for the streamed path)
    eps       : target accuracy of the workload
    name      : label
    """

    x: np.ndarray
    y: np.ndarray
    r: np.ndarray
    c: np.ndarray
    s: float
    cost_scale: float
    C64: np.ndarray | None
    C32: np.ndarray | None
    eps: float
    name: str

    @property
    def n(self) -> int:
        return int(self.r.shape[0])

    @property
    def m(self) -> int:
        return int(self.c.shape[0])


def _rng(cfg: int, k: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([cfg, k])))


def sqeuclid_cost(x32: np.ndarray, y32: np.ndarray):
    """FP64 squared distances between FP32 points, normalised to max 1.

    Returns (C64, scale) with C64 = scale * |x_i - y_j|^2 and
    scale = 1 / max_ij |x_i - y_j|^2.  Computed by differences (not the
    expanded form) so it is accurate to FP64 rounding.
    """
    x = np.asarray(x32, dtype=np.float64)
    y = np.asarray(y32, dtype=np.float64)
    D = np.zeros((x.shape[0], y.shape[0]), dtype=np.float64)
    for k in range(x.shape[1]):
        diff = x[:, k:k + 1] - y[None, :, k]
        D += diff * diff
    mx = float(D.max())
    scale = 1.0 / mx if mx > 0 else 1.0
    return D * scale, scale


def to_bf16_bits(a32: np.ndarray) -> np.ndarray:
    """FP32 -> BF16 by round-to-nearest-even; returns uint16 bit patterns."""
    b = np.ascontiguousarray(a32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    rounded = (b + 0x7FFF + lsb) >> 16
    return rounded.astype(np.uint16)


def bf16_bits_to_f64(bits: np.ndarray) -> np.ndarray:
    """BF16 bit patterns -> exact FP64 values."""
    u32 = bits.astype(np.uint32) << 16
    return u32.view(np.float32).astype(np.float64)


def _finish(x, y, r, c, s, eps, name, dense=True):
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    if dense:
        C64, scale = sqeuclid_cost(x, y)
        C32 = C64.astype(np.float32)
    else:
        C64 = C32 = None
        scale = _max_scale(x, y)
    return Instance(x=x, y=y, r=np.ascontiguousarray(r, dtype=np.float64),
                    c=np.ascontiguousarray(c, dtype=np.float64), s=float(s),
                    cost_scale=float(scale), C64=C64, C32=C32, eps=float(eps), name=name)


def _max_scale(x32, y32, block=2048):
    """1 / max squared distance, blockwise so large clouds fit in memory."""
    x = np.asarray(x32, dtype=np.float64)
    y = np.asarray(y32, dtype=np.float64)
    mx = 0.0
    for i0 in range(0, x.shape[0], block):
        xb = x[i0:i0 + block]
        D = np.zeros((xb.shape[0], y.shape[0]))
        for k in range(x.shape[1]):
            diff = xb[:, k:k + 1] - y[None, :, k]
            D += diff * diff
        mx = max(mx, float(D.max()))
    return 1.0 / mx if mx > 0 else 1.0


def c1(k: int = 0, dense: bool = True) -> Instance:
    """n = m = 100, 2-D uniform points; r ~ Dir(1)*1.0, c ~ Dir(1)*1.2; s = 0.8."""
    g = _rng(1, k)
    x = g.uniform(0.0, 1.0, size=(100, 2))
    y = g.uniform(0.0, 1.0, size=(100, 2))
    r = g.dirichlet(np.ones(100)) * 1.0
    c = g.dirichlet(np.ones(100)) * 1.2
    return _finish(x, y, r, c, 0.8, 1e-2, f"c1[{k}] n=m=100 2-D uniform", dense)


def _cluster_cloud(g, centres, n, sigma, outlier_frac):
    k = centres.shape[0]
    n_out = int(round(outlier_frac * n))
    n_in = n - n_out
    lab = g.integers(0, k, size=n_in)
    pts_in = centres[lab] + sigma * g.standard_normal(size=(n_in, centres.shape[1]))
    pts_out = g.uniform(0.0, 1.0, size=(n_out, centres.shape[1]))
    pts = np.concatenate([pts_in, pts_out], axis=0)
    return pts[g.permutation(n)]


def c2(k: int = 0, n: int = 4096, dense: bool = True) -> Instance:
    """n = m = 4096, 3-D: 8 shared centres ~ U[0,1]^3, 90 % inliers
    centre + N(0, 0.05^2 I), 10 % uniform outliers; uniform masses with totals
    1.0 / 1.0; s = 0.9."""
    g = _rng(2, k)
    centres = g.uniform(0.0, 1.0, size=(8, 3))
    x = _cluster_cloud(g, centres, n, 0.05, 0.10)
    y = _cluster_cloud(g, centres, n, 0.05, 0.10)
    r = np.full(n, 1.0 / n)
    c = np.full(n, 1.0 / n)
    return _finish(x, y, r, c, 0.9, 1e-2, f"c2[{k}] n=m={n} 3-D clusters+outliers", dense)


def tight_clusters(n: int = 512, k: int = 0, sigma: float = 0.01) -> Instance:
    """The recipe of c2() (3-D, 8 clusters, 10 % outliers) with tighter
    clusters (sigma = 0.01 by default): many pairs cost almost nothing, so
    the cold start's total T is large and the first step of a long-step rule
    moves w by thousands (statistics far below the FP64 range at the next
    point).  n = m, uniform masses 1/1, s = 0.9."""
    g = _rng(7, k)
    centres = g.uniform(0.0, 1.0, size=(8, 3))
    x = _cluster_cloud(g, centres, n, sigma, 0.10)
    y = _cluster_cloud(g, centres, n, sigma, 0.10)
    r = np.full(n, 1.0 / n)
    c = np.full(n, 1.0 / n)
    return _finish(x, y, r, c, 0.9, 1e-2, f"tight[{k}] n=m={n} 3-D clusters sigma={sigma}")


def c3(k: int = 0, n: int = 20000, eps: float = 1e-2, dense: bool = True) -> Instance:
    """n = m = 20000, 2-D: source is a 5-component equal-weight Gaussian
    mixture (centres ~ U[0,1]^2, sigma = 0.05); target is the same mixture
    shifted by (0.1, 0.1); uniform masses with totals 1.0 / 1.0; s = 0.7."""
    g = _rng(3, k)
    centres = g.uniform(0.0, 1.0, size=(5, 2))
    lab_x = g.integers(0, 5, size=n)
    lab_y = g.integers(0, 5, size=n)
    x = centres[lab_x] + 0.05 * g.standard_normal(size=(n, 2))
    y = centres[lab_y] + 0.05 * g.standard_normal(size=(n, 2)) + np.array([0.1, 0.1])
    r = np.full(n, 1.0 / n)
    c = np.full(n, 1.0 / n)
    return _finish(x, y, r, c, 0.7, eps, f"c3[{k}] n=m={n} 2-D shifted mixtures", dense)


def _masses_c4(g, n, m):
    r = g.dirichlet(np.full(n, 0.5)) * g.uniform(0.8, 1.2)
    c = g.dirichlet(np.full(m, 0.5)) * g.uniform(0.8, 1.2)
    s = g.uniform(0.5, 0.9) * min(r.sum(), c.sum())
    return r, c, s


def c4_instance(k: int, dense: bool = True) -> Instance:
    """One instance of the uneven batch: n, m = round(exp U(ln 64, ln 1024))
    drawn independently, 3-D uniform points, r, c ~ Dir(0.5) scaled by
    U[0.8, 1.2], s ~ U[0.5, 0.9] * min mass."""
    g = _rng(4, k)
    n = int(round(math.exp(g.uniform(math.log(64), math.log(1024)))))
    m = int(round(math.exp(g.uniform(math.log(64), math.log(1024)))))
    x = g.uniform(0.0, 1.0, size=(n, 3))
    y = g.uniform(0.0, 1.0, size=(m, 3))
    r, c, s = _masses_c4(g, n, m)
    return _finish(x, y, r, c, s, 1e-2, f"c4[{k}] n={n} m={m} 3-D uniform", dense)


def c4_batch(count: int = 512, start: int = 0, dense: bool = True):
    return [c4_instance(k, dense) for k in range(start, start + count)]


def c5(k: int, dense: bool = True) -> Instance:
    """n = m = 256, 2-D Gaussian mixtures: K ~ U{2..5} components, centres
    ~ U[0,1]^2, sigma ~ U[0.03, 0.1] (drawn separately for source and target);
    masses and s as in the uneven batch."""
    g = _rng(5, k)
    n = m = 256

    def mixture(npts):
        kk = int(g.integers(2, 6))
        centres = g.uniform(0.0, 1.0, size=(kk, 2))
        sig = g.uniform(0.03, 0.1)
        lab = g.integers(0, kk, size=npts)
        return centres[lab] + sig * g.standard_normal(size=(npts, 2))

    x = mixture(n)
    y = mixture(m)
    r, c, s = _masses_c4(g, n, m)
    return _finish(x, y, r, c, s, 1e-2, f"c5[{k}] n=m=256 2-D mixtures", dense)


def c5_batch(count: int = 1024, start: int = 30000, dense: bool = True):
    return [c5(k, dense) for k in range(start, start + count)]


def uniform_pair(n: int, m: int, d: int, seed: int, mass_r=1.0, mass_c=1.0,
                 s_frac=0.8, eps=1e-2, dirichlet=1.0) -> Instance:
    """Generic test instance: uniform points in [0,1]^d, Dirichlet masses."""
    g = _rng(100, seed)
    x = g.uniform(0.0, 1.0, size=(n, d))
    y = g.uniform(0.0, 1.0, size=(m, d))
    r = g.dirichlet(np.full(n, dirichlet)) * mass_r
    c = g.dirichlet(np.full(m, dirichlet)) * mass_c
    s = s_frac * min(r.sum(), c.sum())
    return _finish(x, y, r, c, s, eps, f"uniform n={n} m={m} d={d} seed={seed}")


def small_instance(n: int, m: int, seed: int, **kw) -> Instance:
    return uniform_pair(n, m, 2, seed, **kw)


WORKLOADS = {
    "c1": "n=m=100 2-D uniform, Dir(1) masses 1.0/1.2, s=0.8, eps=1e-2",
    "c2": "n=m=4096 3-D 8 clusters + 10% outliers, uniform masses 1/1, s=0.9, eps=1e-2",
    "c3": "n=m=20000 2-D shifted 5-mixtures, uniform masses 1/1, s=0.7, eps in {1e-2, 5e-3}",
    "c4": "512 uneven instances n,m log-uniform [64,1024], 3-D, Dir(0.5) masses",
    "c5": "1024 instances n=m=256 2-D mixtures (warm-start workload)",
}
