"""Seeded generators for the optimal-transport workloads.

Every instance is drawn with ``numpy.random.default_rng(seed)`` (PCG64).  The
cost is either given by coordinates (points or an image grid) or materialised
as a dense FP64 matrix by :meth:`Instance.dense_cost`; the dense form is what
the CPU oracle consumes, the coordinate form is what the GPU may regenerate.

Cost definitions (problem data, eq. ot of the paper; grid costs as in its
Section 5.1 with the squared Euclidean distance):
  points_sqeuclid  C_ij = sum_k (x_ik - y_jk)^2
  points_euclid    C_ij = sqrt(sum_k (x_ik - y_jk)^2)
  grid_sqeuclid    C_ij = h * ((a_i - a_j)^2 + (b_i - b_j)^2), pixel i = (a_i, b_i) =
                   (i // s, i % s) on an s x s image, h = 1 / (2 (s-1)^2) so max C = 1
  grid_l1 / grid_l2 / grid_linf  the Section 5.1 pixel-distance costs times h1 = 1/(s-1)
The sums over k run in index order in FP64, the grid product is one FP64 multiply.
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Instance:
    m: int
    n: int
    f: np.ndarray
    g: np.ndarray
    kind: str
    x: Optional[np.ndarray] = None      # m x d source coordinates (points kinds)
    y: Optional[np.ndarray] = None      # n x d target coordinates
    side: int = 0                       # grid kinds: image side s (m = n = s*s)
    scale: float = 1.0                  # grid kinds: h
    tol: float = 1e-6
    meta: dict = field(default_factory=dict)

    def dense_cost(self) -> np.ndarray:
        """FP64 m x n cost matrix."""
        if self.kind in ("points_sqeuclid", "points_euclid"):
            d = self.x.shape[1]
            C = np.zeros((self.m, self.n))
            for k in range(d):
                diff = self.x[:, k][:, None] - self.y[:, k][None, :]
                C = C + diff * diff
            if self.kind == "points_euclid":
                C = np.sqrt(C)
            return C
        if self.kind.startswith("grid_"):
            s = self.side
            idx = np.arange(s * s)
            a = (idx // s).astype(np.float64)
            b = (idx % s).astype(np.float64)
            da = a[:, None] - a[None, :]
            db = b[:, None] - b[None, :]
            if self.kind == "grid_sqeuclid":
                return (da * da + db * db) * self.scale
            if self.kind == "grid_l1":
                return (np.abs(da) + np.abs(db)) * self.scale
            if self.kind == "grid_l2":
                return np.sqrt(da * da + db * db) * self.scale
            if self.kind == "grid_linf":
                return np.maximum(np.abs(da), np.abs(db)) * self.scale
        if self.kind == "dense":
            return self.meta["C"]
        raise ValueError(self.kind)


def _normalise(w):
    w = np.asarray(w, dtype=np.float64)
    return w / w.sum()


def points_sqeuclid(seed: int, m: int = 64, n: int = 64, dim: int = 2, tol: float = 1e-6):
    """Uniform points in [0,1]^dim, weights U(0.1,1) normalised (drawn in the order
    src points, tgt points, f, g)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, size=(m, dim))
    y = rng.uniform(0.0, 1.0, size=(n, dim))
    f = _normalise(rng.uniform(0.1, 1.0, size=m))
    g = _normalise(rng.uniform(0.1, 1.0, size=n))
    return Instance(m, n, f, g, "points_sqeuclid", x=x, y=y, tol=tol, meta={"seed": seed})


def blob_histogram(rng, s: int, blobs: int = 5, floor: float = 1e-3):
    """Sum of Gaussian blobs on an s x s image: centre U[0,s-1]^2, sigma U(0.05s,0.25s),
    amplitude U(0.2,1); then H/max(H) + floor, normalised to sum 1 (row-major)."""
    a = np.arange(s, dtype=np.float64)
    A, B = np.meshgrid(a, a, indexing="ij")
    H = np.zeros((s, s))
    for _ in range(blobs):
        ca, cb = rng.uniform(0.0, s - 1.0, size=2)
        sig = rng.uniform(0.05 * s, 0.25 * s)
        amp = rng.uniform(0.2, 1.0)
        H += amp * np.exp(-((A - ca) ** 2 + (B - cb) ** 2) / (2.0 * sig * sig))
    H = H / H.max() + floor
    return _normalise(H.reshape(-1))


def grid_pair(seed: int, side: int, kind: str = "grid_sqeuclid", tol: float = 1e-6):
    """Two s x s blob histograms and a pixel-distance cost scaled so max C = 1
    (stand-in for the paper's DOTmark image pairs, which are not available)."""
    rng = np.random.default_rng(seed)
    f = blob_histogram(rng, side)
    g = blob_histogram(rng, side)
    if kind == "grid_sqeuclid":
        h = 1.0 / (2.0 * (side - 1) ** 2)
    elif kind == "grid_l1":
        h = 1.0 / (2.0 * (side - 1))
    elif kind == "grid_l2":
        h = 1.0 / (np.sqrt(2.0) * (side - 1))
    elif kind == "grid_linf":
        h = 1.0 / (side - 1)
    else:
        raise ValueError(kind)
    mm = side * side
    return Instance(mm, mm, f, g, kind, side=side, scale=h, tol=tol,
                    meta={"seed": seed})


# ---- synthetic image classes standing in for the DOTmark classes (Section 5.1), which are
# not available; each returns a nonnegative s x s image, normalised to sum 1 (row-major)

IMAGE_CLASSES = ("blobs", "white_noise", "cauchy", "smooth_field", "shapes")


def class_image(rng, s: int, cls: str, floor: float = 1e-3):
    a = np.arange(s, dtype=np.float64)
    A, B = np.meshgrid(a, a, indexing="ij")
    if cls == "blobs":
        return blob_histogram(rng, s, floor=floor)
    if cls == "white_noise":
        H = rng.uniform(0.0, 1.0, size=(s, s))
    elif cls == "cauchy":
        # sum of three Cauchy bumps (heavy tails), widths U(0.02s, 0.2s)
        H = np.zeros((s, s))
        for _ in range(3):
            ca, cb = rng.uniform(0.0, s - 1.0, size=2)
            w = rng.uniform(0.02 * s, 0.2 * s)
            H += 1.0 / (1.0 + ((A - ca) ** 2 + (B - cb) ** 2) / (w * w))
    elif cls == "smooth_field":
        # Gaussian random field: white noise filtered by a Gaussian of width s/8 (periodic)
        k = np.fft.fftfreq(s)
        K2 = k[:, None] ** 2 + k[None, :] ** 2
        spec = np.fft.fft2(rng.normal(size=(s, s))) * np.exp(-2.0 * (np.pi * s / 8.0) ** 2 * K2)
        H = np.real(np.fft.ifft2(spec))
        H = np.exp(2.0 * H / H.std())          # log-normal field, positive
    elif cls == "shapes":
        # up to four filled rectangles and discs
        H = np.zeros((s, s))
        for _ in range(int(rng.integers(2, 5))):
            ca, cb = rng.uniform(0.0, s - 1.0, size=2)
            r = rng.uniform(0.05 * s, 0.25 * s)
            if rng.uniform() < 0.5:
                H += ((A - ca) ** 2 + (B - cb) ** 2 <= r * r)
            else:
                H += (np.abs(A - ca) <= r) & (np.abs(B - cb) <= 0.6 * r)
    else:
        raise ValueError(cls)
    H = H / H.max() + floor
    return _normalise(H.reshape(-1))


def suite_pair(seed: int, side: int, cls: str, norm: str, tol: float = 1e-4):
    """Two images of one class and the raw pixel distance of the given norm (C^1, C^2 or
    C^inf of Section 5.1, not rescaled)."""
    rng = np.random.default_rng(seed)
    f = class_image(rng, side, cls)
    g = class_image(rng, side, cls)
    kind = {"l1": "grid_l1", "l2": "grid_l2", "linf": "grid_linf"}[norm]
    mm = side * side
    return Instance(mm, mm, f, g, kind, side=side, scale=1.0, tol=tol,
                    meta={"seed": seed, "class": cls, "norm": norm})


def gmm_points(rng, count: int, dim: int = 3, comps: int = 3):
    means = rng.normal(0.0, 2.0, size=(comps, dim))
    stds = rng.uniform(0.3, 1.0, size=comps)
    lab = rng.integers(0, comps, size=count)
    return means[lab] + stds[lab][:, None] * rng.normal(size=(count, dim))


def gmm_euclid(seed: int, m: int, n: int, tol: float = 1e-4):
    """3-component Gaussian mixtures in R^3 (weights 1/3, means N(0,4I), isotropic
    std U(0.3,1)), drawn separately for source and target; Euclidean cost;
    marginals LogNormal(0,1) normalised."""
    rng = np.random.default_rng(seed)
    x = gmm_points(rng, m)
    y = gmm_points(rng, n)
    f = _normalise(rng.lognormal(0.0, 1.0, size=m))
    g = _normalise(rng.lognormal(0.0, 1.0, size=n))
    return Instance(m, n, f, g, "points_euclid", x=x, y=y, tol=tol, meta={"seed": seed})


def log_uniform_int(rng, lo: int, hi: int) -> int:
    return int(round(float(np.exp(rng.uniform(np.log(lo), np.log(hi))))))


def batch_instances(count: int = 256, master_seed: int = 300, lo: int = 32, hi: int = 2048,
                    tol: float = 1e-4):
    """Uneven batch: m, n log-uniform in [lo, hi] independently; instance i uses seed
    1000*master_seed + i."""
    rng = np.random.default_rng(master_seed)
    sizes = [(log_uniform_int(rng, lo, hi), log_uniform_int(rng, lo, hi)) for _ in range(count)]
    return [gmm_euclid(1000 * master_seed + i, m, n, tol=tol) for i, (m, n) in enumerate(sizes)]


def serving_stream(count: int = 2000, master_seed: int = 500, rate: float = 10.0,
                   lo: int = 64, hi: int = 16384, grid_fraction: float = 0.1,
                   grid_lo: int = 8, grid_hi: int = 128, tols=(1e-4, 1e-6)):
    """Poisson request stream: exponential inter-arrival times at `rate` requests/s.
    90% point-cloud pairs (U[0,1]^2, weights U(0.1,1), squared Euclidean), 10% blob-grid
    pairs with side log-uniform in [grid_lo, grid_hi]; tolerance drawn from `tols`.
    Returns a list of (arrival_time_s, Instance)."""
    rng = np.random.default_rng(master_seed)
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate))
        tol = float(tols[int(rng.integers(0, len(tols)))])
        seed = 1000 * master_seed + i
        if rng.uniform() < grid_fraction:
            s = log_uniform_int(rng, grid_lo, grid_hi)
            inst = grid_pair(seed, s, tol=tol)
        else:
            m = log_uniform_int(rng, lo, hi)
            n = log_uniform_int(rng, lo, hi)
            inst = points_sqeuclid(seed, m, n, tol=tol)
        out.append((t, inst))
    return out


def config_instance(config: int, index: int = 0):
    """The fixed single-instance workloads: 1 -> 64x64 points, 2 -> 32x32 grids (1024),
    3 -> 64x64 grids (4096)."""
    if config == 1:
        return points_sqeuclid(index, 64, 64, tol=1e-6)
    if config == 2:
        return grid_pair(100 + index, 32, tol=1e-6)
    if config == 3:
        return grid_pair(200 + index, 64, tol=1e-6)
    raise ValueError(config)
