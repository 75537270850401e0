"""Seeded synthetic inputs shaped like the paper's AIDW workloads.

The paper times AIDW on m = n points placed at random in a square, at sizes
10K..1000K with 1K = 1024 (Sec. 4).  It uses no public dataset; the
generators below stand in for its inputs and add a clustered, a batched and a
served variant.  This module draws random numbers and packs arrays only: it
holds none of the interpolation arithmetic, and both the oracle and the HIP
path consume exactly the arrays it returns.

Draw order per instance: data x, data y, data z noise (or the mixture draws),
then the queries.  Coordinates and values are generated in float64 and, for
FP32 workloads, rounded to float32 once; the oracle promotes those same
rounded values.  The study area A of Eq. 2 is the float64 area of the data
points' bounding box.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

LEVELS = (1.0, 2.0, 3.0, 4.0, 5.0)


@dataclass
class Instance:
    """One AIDW problem: m data points (x, y, z) and n queries (x, y)."""

    name: str
    data_x: np.ndarray
    data_y: np.ndarray
    data_z: np.ndarray
    query_x: np.ndarray
    query_y: np.ndarray
    k: int
    area: float
    levels: tuple = LEVELS
    R_min: float = 0.0
    R_max: float = 2.0
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.data_x.shape[0])

    @property
    def n(self) -> int:
        return int(self.query_x.shape[0])

    @property
    def dtype(self):
        return self.data_x.dtype

    def data_xy(self) -> np.ndarray:
        """Planar [2, m] array: the x row, then the y row."""
        return np.ascontiguousarray(np.stack([self.data_x, self.data_y]))

    def query_xy(self) -> np.ndarray:
        """Planar [2, n] array: the x row, then the y row."""
        return np.ascontiguousarray(np.stack([self.query_x, self.query_y]))

    def pair_evals(self) -> int:
        """Distance evaluations of both full passes: 2 * m * n."""
        return 2 * self.m * self.n


def bbox_area(x: np.ndarray, y: np.ndarray) -> float:
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return float((x.max() - x.min()) * (y.max() - y.min()))


def _cast(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(dtype))


def _finish(name, x, y, z, qx, qy, k, dtype, meta=None, levels=LEVELS):
    x, y, z = _cast(x, dtype), _cast(y, dtype), _cast(z, dtype)
    qx, qy = _cast(qx, dtype), _cast(qy, dtype)
    return Instance(name, x, y, z, qx, qy, int(k), bbox_area(x, y), tuple(levels),
                    meta=dict(meta or {}))


def uniform_small(m=1024, n=1024, seed=0, k=10, dtype=np.float64):
    """m data and n query points U[0,1]^2, z = sin(4x)cos(3y) + N(0, 0.01^2).

    At m = n = 1024, k = 10, seed 0 this is the small plain-AIDW workload
    (FP64, single instance)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, m)
    y = rng.uniform(0.0, 1.0, m)
    z = np.sin(4.0 * x) * np.cos(3.0 * y) + rng.normal(0.0, 0.01, m)
    qx = rng.uniform(0.0, 1.0, n)
    qy = rng.uniform(0.0, 1.0, n)
    return _finish("uniform_small_m%d_n%d" % (m, n), x, y, z, qx, qy, k, dtype,
                   {"seed": seed})


def paper_scale(m=1 << 20, n=1 << 20, seed=1, k=15, dtype=np.float32):
    """m data and n query points U[0,1000]^2,
    z = 0.01x + 0.02y + 5 sin(x/50) + N(0, 1).

    At m = n = 2^20, k = 15 this is the paper-scale single instance (the
    paper's largest size is 1000K = 1,024,000 points in a square)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1000.0, m)
    y = rng.uniform(0.0, 1000.0, m)
    z = 0.01 * x + 0.02 * y + 5.0 * np.sin(x / 50.0) + rng.normal(0.0, 1.0, m)
    qx = rng.uniform(0.0, 1000.0, n)
    qy = rng.uniform(0.0, 1000.0, n)
    return _finish("paper_scale_m%d_n%d" % (m, n), x, y, z, qx, qy, k, dtype, {"seed": seed})


def _mixture_points(rng, count, centres, sigmas):
    """`count` points from an equal-weight isotropic Gaussian mixture in
    [0,1]^2; draws that fall outside the square are drawn again."""
    comp = rng.integers(0, centres.shape[0], count)
    pts = centres[comp] + rng.normal(0.0, 1.0, (count, 2)) * sigmas[comp, None]
    bad = np.nonzero((pts < 0.0).any(axis=1) | (pts > 1.0).any(axis=1))[0]
    while bad.size:
        c = comp[bad]
        pts[bad] = centres[c] + rng.normal(0.0, 1.0, (bad.size, 2)) * sigmas[c, None]
        bad = bad[(pts[bad] < 0.0).any(axis=1) | (pts[bad] > 1.0).any(axis=1)]
    return pts


def clustered(m=1 << 18, n=1 << 18, seed=2, k=10, dtype=np.float32, n_centres=64,
              background=0.10, on_point=0.01):
    """Clustered precision stress.

    Data: (1 - background) of the points from a 64-component isotropic
    Gaussian mixture (centres U[0,1]^2, equal weights, sigma log-uniform in
    [1e-4, 1e-1]), the rest U[0,1]^2.  Queries U[0,1]^2, then a fraction
    `on_point` of them overwritten with exact copies of random data points.
    z = sum over the centres c of exp(-10 |p - c|^2)."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, (n_centres, 2))
    sigmas = np.exp(rng.uniform(np.log(1e-4), np.log(1e-1), n_centres))
    n_mix = int(round((1.0 - background) * m))
    pts = np.empty((m, 2))
    pts[:n_mix] = _mixture_points(rng, n_mix, centres, sigmas)
    pts[n_mix:] = rng.uniform(0.0, 1.0, (m - n_mix, 2))
    pts = pts[rng.permutation(m)]
    z = np.zeros(m)
    for c in centres:
        z += np.exp(-10.0 * ((pts[:, 0] - c[0]) ** 2 + (pts[:, 1] - c[1]) ** 2))
    x, y = pts[:, 0], pts[:, 1]
    qx = rng.uniform(0.0, 1.0, n)
    qy = rng.uniform(0.0, 1.0, n)
    n_on = int(round(on_point * n))
    on_q = rng.choice(n, n_on, replace=False) if n_on else np.zeros(0, dtype=np.int64)
    on_d = rng.integers(0, m, n_on)
    # copy after the FP32 rounding so the copies are exact in the stored dtype
    inst = _finish("clustered_m%d_n%d" % (m, n), x, y, z, qx, qy, k, dtype, {"seed": seed})
    inst.query_x[on_q] = inst.data_x[on_d]
    inst.query_y[on_q] = inst.data_y[on_d]
    inst.meta["on_point_queries"] = np.sort(on_q)
    inst.meta["on_point_data"] = on_d[np.argsort(on_q)]
    return inst


def _log_uniform_int(rng, lo, hi, size=None):
    return np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size))).astype(np.int64)


def batched(count=512, seed=3, m_range=(1024, 65536), n_range=(1024, 32768),
            ks=(8, 10, 15), dtype=np.float32):
    """`count` independent instances of uneven size for one batched launch:
    m and n log-uniform in the given ranges, uniform or clustered points with
    probability 1/2 each, k drawn from `ks`."""
    rng = np.random.default_rng(seed)
    ms = _log_uniform_int(rng, *m_range, count)
    ns = _log_uniform_int(rng, *n_range, count)
    kinds = rng.integers(0, 2, count)
    kk = rng.choice(np.asarray(ks), count)
    subseeds = rng.integers(0, 2**31 - 1, count)
    out = []
    for i in range(count):
        if kinds[i] == 0:
            inst = uniform_unit(int(ms[i]), int(ns[i]), int(subseeds[i]), int(kk[i]), dtype)
        else:
            inst = clustered(int(ms[i]), int(ns[i]), int(subseeds[i]), int(kk[i]), dtype,
                             on_point=0.0)
        inst.name = "batch%03d_%s" % (i, inst.name)
        out.append(inst)
    return out


def dense_patch(m=16384, n=2048, seed=5, k=15, dtype=np.float32, patch_frac=0.3,
                patch_queries=0.25):
    """U[0,1]^2 data with a fraction `patch_frac` of the points moved into the
    square [0.45, 0.55]^2 (forty times the background density there), and
    queries: the first `patch_queries` of them inside that square, the rest
    U[0,1]^2.  Queries in the patch have far nearer neighbours than m points
    spread over the bounding box would give, so R falls below R_max there and
    alpha below alpha_5; elsewhere alpha is alpha_5 for nearly every query.
    z = sin(4x)cos(3y) + N(0, 0.01^2)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, m)
    y = rng.uniform(0.0, 1.0, m)
    z_noise = rng.normal(0.0, 0.01, m)
    n_patch = int(round(patch_frac * m))
    x[:n_patch] = rng.uniform(0.45, 0.55, n_patch)
    y[:n_patch] = rng.uniform(0.45, 0.55, n_patch)
    z = np.sin(4.0 * x) * np.cos(3.0 * y) + z_noise
    qx = rng.uniform(0.0, 1.0, n)
    qy = rng.uniform(0.0, 1.0, n)
    nq = int(round(patch_queries * n))
    qx[:nq] = rng.uniform(0.45, 0.55, nq)
    qy[:nq] = rng.uniform(0.45, 0.55, nq)
    return _finish("dense_patch_m%d_n%d" % (m, n), x, y, z, qx, qy, k, dtype, {"seed": seed})


def uniform_unit(m, n, seed, k, dtype=np.float32):
    """m data and n query points U[0,1]^2, z = sin(4x)cos(3y) + N(0, 0.01^2)."""
    inst = uniform_small(m, n, seed, k, dtype)
    inst.name = "uniform_m%d_n%d" % (m, n)
    return inst


@dataclass
class Request:
    t_arrival: float
    dataset: int
    n: int
    k: int
    query_seed: int


def serving_stream(count=10000, rate=2000.0, seed=4, m_range=(4096, 1 << 20),
                   n_range=(256, 1 << 18), ks=(8, 10, 15), reuse=0.20):
    """Poisson arrivals of AIDW jobs.  Each request names a dataset (a data
    point set of log-uniform size m, uniform or clustered) and draws its own
    queries; a fraction `reuse` of requests reuse an earlier dataset.
    Returns (requests, dataset_specs) where dataset_specs[i] = (m, kind, seed);
    the arrays are drawn on demand with `dataset_arrays`/`request_queries`."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, count)
    t = np.cumsum(gaps)
    datasets = []
    reqs = []
    for i in range(count):
        if datasets and rng.uniform() < reuse:
            ds = int(rng.integers(0, len(datasets)))
        else:
            m = int(_log_uniform_int(rng, *m_range))
            datasets.append((m, int(rng.integers(0, 2)), int(rng.integers(0, 2**31 - 1))))
            ds = len(datasets) - 1
        n = int(_log_uniform_int(rng, *n_range))
        k = int(rng.choice(np.asarray(ks)))
        reqs.append(Request(float(t[i]), ds, n, k, int(rng.integers(0, 2**31 - 1))))
    return reqs, datasets


def dataset_arrays(spec, dtype=np.float32):
    """(x, y, z, area) of a serving dataset spec (m, kind, seed)."""
    m, kind, seed = spec
    if kind == 0:
        inst = uniform_unit(m, 1, seed, 1, dtype)
    else:
        inst = clustered(m, 1, seed, 1, dtype, on_point=0.0)
    return inst.data_x, inst.data_y, inst.data_z, inst.area


def request_queries(req: Request, dtype=np.float32):
    rng = np.random.default_rng(req.query_seed)
    qx = rng.uniform(0.0, 1.0, req.n)
    qy = rng.uniform(0.0, 1.0, req.n)
    return _cast(qx, dtype), _cast(qy, dtype)


def hand_points(points, values, queries, dtype=np.float64):
    """Pack small hand-written examples into arrays."""
    p = np.asarray(points, dtype=np.float64).reshape(-1, 2)
    q = np.asarray(queries, dtype=np.float64).reshape(-1, 2)
    z = np.asarray(values, dtype=np.float64)
    return (_cast(p[:, 0], dtype), _cast(p[:, 1], dtype), _cast(z, dtype),
            _cast(q[:, 0], dtype), _cast(q[:, 1], dtype))
