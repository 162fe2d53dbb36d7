"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random point sets and masses; it contains none of the
method's arithmetic and imports neither the GPU library nor the oracle, so
both sides of every parity test read the very same values from it.

Conventions (shared by every workload):
  * numpy ``Generator(PCG64(seed))``; pair / set ``p`` of a workload draws
    from ``SeedSequence([seed, p])`` so any subset can be regenerated alone;
  * values are sampled in FP64 and rounded to FP32 (round-to-nearest-even);
    the BF16 workload rounds the FP32 values to BF16 the same way;
  * masses are normalised in FP64 and then rounded to FP32, without
    renormalising afterwards (so the two totals differ by FP32 rounding);
  * integer sizes are drawn inclusive of both ends.

Workloads (the suppliers X,a are searched by the consumers Y,b):
  single_pair_2d     n = m = 256, U[0,1]^2, uniform masses 1/256, L2.
  batched_hist_3d    P pairs, m, n ~ U{128..1024} independently, U[0,1]^3
                     (a colour/intensity histogram stand-in), Dirichlet(1)
                     masses, L2.
  documents_300d     1 query vs C candidates, sizes ~ U{20..500},
                     N(0,1)/sqrt(300) in 300-d stored as BF16, Zipf(1.1)
                     rank-frequency masses, L2 (a word-embedding stand-in).
  colour_transfer_3d n = m = 65536, two-component Gaussian mixture per side
                     clipped to [0,1]^3, uniform masses, squared Euclidean.
  retrieval_3d       1 query vs C candidates of 256 points each, Gaussian
                     mixtures with 1..8 components, uniform masses.
  lattice_hist_2d    N images on an s x s pixel grid (s = 28 or 32): every
                     pixel is a point at its integer (row, col), its mass the
                     normalised 8-bit intensity; pair p = (image p, image
                     p + 1 mod N), L2.  Two image styles: sparse strokes
                     (digit-like, most pixels 0) and smooth positive
                     densities (sums of Gaussian bumps).
  colour_images      seeded smooth RGB images (8-bit) for the colour
                     transfer application.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEEDS = {
    "single_pair_2d": 1001,
    "batched_hist_3d": 1002,
    "documents_300d": 1003,
    "colour_transfer_3d": 1004,
    "retrieval_3d": 1005,
    "lattice_hist_2d": 1006,
    "colour_images": 1007,
}


def rng_for(seed: int, p: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, p])))


def to_f32(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def f32_to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round FP32 values to BF16 (round-to-nearest-even); returns uint16 bits."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    rounded = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return rounded.astype(np.uint16)


def bf16_bits_to_f32(bits: np.ndarray) -> np.ndarray:
    return (np.asarray(bits, dtype=np.uint32) << 16).view(np.float32)


@dataclass
class PairSet:
    """Concatenated ragged point sets plus the pairs to compare.

    X (num_x_rows x d) with masses a and set offsets x_off (len num_x_sets+1);
    likewise Y, b, y_off.  Pair p compares X-set pair_x[p] (suppliers) with
    Y-set pair_y[p] (consumers); None means pair p = (p, p).
    ``X_bits``/``Y_bits`` hold BF16 storage when the workload is BF16 (then
    X/Y are the exact FP32 values of those BF16 numbers).
    """
    name: str
    d: int
    X: np.ndarray
    a: np.ndarray
    x_off: np.ndarray
    Y: np.ndarray
    b: np.ndarray
    y_off: np.ndarray
    pair_x: np.ndarray | None = None
    pair_y: np.ndarray | None = None
    metric: str = "l2"
    dtype: str = "f32"
    X_bits: np.ndarray | None = None
    Y_bits: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def num_pairs(self) -> int:
        return len(self.pair_x) if self.pair_x is not None else len(self.x_off) - 1

    def pair(self, p: int):
        """(X_p, a_p, Y_p, b_p) views of pair p."""
        px = int(self.pair_x[p]) if self.pair_x is not None else p
        py = int(self.pair_y[p]) if self.pair_y is not None else p
        xs, xe = self.x_off[px], self.x_off[px + 1]
        ys, ye = self.y_off[py], self.y_off[py + 1]
        return self.X[xs:xe], self.a[xs:xe], self.Y[ys:ye], self.b[ys:ye]

    def sizes(self):
        px = self.pair_x if self.pair_x is not None else np.arange(self.num_pairs)
        py = self.pair_y if self.pair_y is not None else np.arange(self.num_pairs)
        m = (self.x_off[1:] - self.x_off[:-1])[px]
        n = (self.y_off[1:] - self.y_off[:-1])[py]
        return m.astype(np.int64), n.astype(np.int64)


def _concat(sets, d):
    if sets:
        pts = np.concatenate([s[0] for s in sets]).reshape(-1, d)
        ms = np.concatenate([s[1] for s in sets])
    else:
        pts = np.zeros((0, d), np.float32)
        ms = np.zeros((0,), np.float32)
    off = np.zeros(len(sets) + 1, np.int64)
    off[1:] = np.cumsum([len(s[1]) for s in sets])
    return np.ascontiguousarray(pts), np.ascontiguousarray(ms), off


def uniform_masses(n: int) -> np.ndarray:
    return to_f32(np.full(n, 1.0 / n)) if n > 0 else np.zeros(0, np.float32)


def dirichlet_masses(rng, n: int) -> np.ndarray:
    """Dirichlet(1) masses: normalised Exp(1) draws (FP64), cast to FP32."""
    e = rng.standard_exponential(n)
    return to_f32(e / e.sum())


def zipf_masses(rng, n: int, s: float = 1.1) -> np.ndarray:
    """Rank-frequency weights k^-s (k = 1..n) in a seeded random order."""
    w = np.arange(1, n + 1, dtype=np.float64) ** (-s)
    w = w / w.sum()
    return to_f32(rng.permutation(w))


def single_pair_2d(n: int = 256, seed: int = SEEDS["single_pair_2d"]) -> PairSet:
    rx, ry = rng_for(seed, 0), rng_for(seed, 1)
    X = to_f32(rx.random((n, 2)))
    Y = to_f32(ry.random((n, 2)))
    a = uniform_masses(n)
    b = uniform_masses(n)
    Xc, ac, xo = _concat([(X, a)], 2)
    Yc, bc, yo = _concat([(Y, b)], 2)
    return PairSet("single_pair_2d", 2, Xc, ac, xo, Yc, bc, yo, metric="l2",
                   meta={"n": n, "seed": seed})


def batched_hist_3d(num_pairs: int = 4096, lo: int = 128, hi: int = 1024,
                    seed: int = SEEDS["batched_hist_3d"]) -> PairSet:
    xs, ys = [], []
    for p in range(num_pairs):
        r = rng_for(seed, p)
        m = int(r.integers(lo, hi + 1))
        n = int(r.integers(lo, hi + 1))
        X = to_f32(r.random((m, 3)))
        Y = to_f32(r.random((n, 3)))
        xs.append((X, dirichlet_masses(r, m)))
        ys.append((Y, dirichlet_masses(r, n)))
    Xc, ac, xo = _concat(xs, 3)
    Yc, bc, yo = _concat(ys, 3)
    return PairSet("batched_hist_3d", 3, Xc, ac, xo, Yc, bc, yo, metric="l2",
                   meta={"num_pairs": num_pairs, "lo": lo, "hi": hi, "seed": seed})


def _doc(r, lo, hi, d):
    k = int(r.integers(lo, hi + 1))
    pts = to_f32(r.standard_normal((k, d)) / np.sqrt(d))
    bits = f32_to_bf16_bits(pts)
    return bits, zipf_masses(r, k)


def documents_300d(num_candidates: int = 8192, lo: int = 20, hi: int = 500, d: int = 300,
                   seed: int = SEEDS["documents_300d"]) -> PairSet:
    """Query = suppliers (set 0 of X); candidate c = consumers (set c of Y)."""
    qb, qa = _doc(rng_for(seed, 0), lo, hi, d)
    cands = [_doc(rng_for(seed, 1 + c), lo, hi, d) for c in range(num_candidates)]
    Xbits, ac, xo = _concat([(qb, qa)], d)
    Ybits, bc, yo = _concat(cands, d)
    ps = PairSet("documents_300d", d, bf16_bits_to_f32(Xbits).reshape(-1, d), ac, xo,
                 bf16_bits_to_f32(Ybits).reshape(-1, d), bc, yo,
                 pair_x=np.zeros(num_candidates, np.int32),
                 pair_y=np.arange(num_candidates, dtype=np.int32),
                 metric="l2", dtype="bf16", X_bits=Xbits.reshape(-1, d),
                 Y_bits=Ybits.reshape(-1, d),
                 meta={"num_candidates": num_candidates, "lo": lo, "hi": hi, "seed": seed})
    return ps


def _gmm_cloud(r, n, k, mean_lo, mean_hi, sig_lo, sig_hi, weights, clip):
    means = r.uniform(mean_lo, mean_hi, size=(k, 3))
    sig = r.uniform(sig_lo, sig_hi, size=k)
    comp = r.choice(k, size=n, p=weights)
    pts = means[comp] + r.standard_normal((n, 3)) * sig[comp, None]
    if clip:
        pts = np.clip(pts, 0.0, 1.0)
    return to_f32(pts)


def colour_transfer_3d(n: int = 65536, seed: int = SEEDS["colour_transfer_3d"]) -> PairSet:
    """Two equal-weight isotropic components per side, means U[0.25,0.75]^3,
    sigma U[0.05,0.15], clipped to [0,1]^3 (clipping makes exact duplicates)."""
    sets = []
    for side in range(2):
        r = rng_for(seed, side)
        pts = _gmm_cloud(r, n, 2, 0.25, 0.75, 0.05, 0.15, np.array([0.5, 0.5]), True)
        sets.append((pts, uniform_masses(n)))
    Xc, ac, xo = _concat([sets[0]], 3)
    Yc, bc, yo = _concat([sets[1]], 3)
    return PairSet("colour_transfer_3d", 3, Xc, ac, xo, Yc, bc, yo, metric="sqeuclidean",
                   meta={"n": n, "seed": seed})


def retrieval_clouds(r, count: int, n: int = 256) -> np.ndarray:
    """count Gaussian-mixture clouds of n 3-D points, shape (count, n, 3):
    K ~ U{1..8} components, means U[0,1]^3, isotropic sigma U[0.02,0.2],
    Dirichlet(1) component weights, no clipping."""
    K = r.integers(1, 9, size=count)
    means = r.uniform(0.0, 1.0, size=(count, 8, 3))
    sig = r.uniform(0.02, 0.2, size=(count, 8))
    w = r.standard_exponential((count, 8)) * (np.arange(8)[None, :] < K[:, None])
    w = w / w.sum(axis=1, keepdims=True)
    cw = np.cumsum(w, axis=1)
    u = r.random((count, n))
    comp = np.minimum((u[:, :, None] >= cw[:, None, :]).sum(axis=2), K[:, None] - 1)
    rows = np.arange(count)[:, None]
    pts = means[rows, comp] + r.standard_normal((count, n, 3)) * sig[rows, comp][..., None]
    return to_f32(pts)


def retrieval_3d(num_candidates: int = 100000, points: int = 256, query: int = 0,
                 seed: int = SEEDS["retrieval_3d"]) -> PairSet:
    """Query q (suppliers) against every candidate (consumers).  Candidates
    come in blocks of 4096 drawn from stream 1_000_000 + block; query q from
    stream q.  Uniform masses."""
    qx = retrieval_clouds(rng_for(seed, query), 1, points)[0]
    blocks = [retrieval_clouds(rng_for(seed, 1_000_000 + k), min(4096, num_candidates - 4096 * k), points)
              for k in range((num_candidates + 4095) // 4096)]
    Y = np.concatenate(blocks).reshape(-1, 3) if blocks else np.zeros((0, 3), np.float32)
    b = np.tile(uniform_masses(points), num_candidates)
    y_off = np.arange(num_candidates + 1, dtype=np.int64) * points
    Xc, ac, xo = _concat([(qx, uniform_masses(points))], 3)
    return PairSet("retrieval_3d", 3, Xc, ac, xo, np.ascontiguousarray(Y), b, y_off,
                   pair_x=np.zeros(num_candidates, np.int32),
                   pair_y=np.arange(num_candidates, dtype=np.int32), metric="l2",
                   meta={"num_candidates": num_candidates, "points": points, "query": query,
                         "seed": seed})


def retrieval_query(query: int, points: int = 256, seed: int = SEEDS["retrieval_3d"]) -> np.ndarray:
    """The query cloud q of retrieval_3d (stream q)."""
    return retrieval_clouds(rng_for(seed, query), 1, points)[0]


def surrogate_training_pairs(num_pairs: int, points: int = 256, seed: int = SEEDS["retrieval_3d"]):
    """Training pairs for the surrogate, drawn like the retrieval clouds from
    streams 2_000_000 + block (disjoint from queries and candidates):
    returns (X, a, set_off) with pair b = (set 2b, set 2b+1)."""
    sets = 2 * num_pairs
    blocks = [retrieval_clouds(rng_for(seed, 2_000_000 + k), min(4096, sets - 4096 * k), points)
              for k in range((sets + 4095) // 4096)]
    X = np.concatenate(blocks).reshape(-1, 3) if blocks else np.zeros((0, 3), np.float32)
    a = np.tile(uniform_masses(points), sets)
    off = np.arange(sets + 1, dtype=np.int64) * points
    return np.ascontiguousarray(X), a, off


def random_pair(seed: int, m: int, n: int, d: int, masses: str = "dirichlet",
                lattice: int = 0) -> tuple:
    """Small seeded pair for tests.  lattice > 0 draws integer coordinates in
    [0, lattice) (exact in FP32, so ties are real).  masses: 'dirichlet',
    'uniform' or 'integer' (small integers normalised, exact-ish ties)."""
    r = rng_for(seed, 0)
    if lattice > 0:
        X = to_f32(r.integers(0, lattice, size=(m, d)))
        Y = to_f32(r.integers(0, lattice, size=(n, d)))
    else:
        X = to_f32(r.random((m, d)))
        Y = to_f32(r.random((n, d)))
    if masses == "uniform":
        a, b = uniform_masses(m), uniform_masses(n)
    elif masses == "integer":
        ia = r.integers(1, 5, size=m).astype(np.float64)
        ib = r.integers(1, 5, size=n).astype(np.float64)
        a, b = to_f32(ia / ia.sum()), to_f32(ib / ib.sum())
    else:
        a, b = dirichlet_masses(r, m), dirichlet_masses(r, n)
    return X, a, Y, b


def random_doc_pair(seed: int, m: int, n: int, d: int, masses: str = "zipf", lattice: int = 0) -> tuple:
    """Small seeded high-dimensional pair for tests, as BF16 bits:
    (X_bits m x d, a, Y_bits n x d, b).  Coordinates N(0,1)/sqrt(d) rounded
    to BF16, or integers in [0, lattice) (exact in BF16 up to 256, so ties
    are real).  masses: 'zipf', 'dirichlet' or 'uniform'."""
    r = rng_for(seed, 0)
    if lattice > 0:
        X = f32_to_bf16_bits(to_f32(r.integers(0, lattice, size=(m, d))))
        Y = f32_to_bf16_bits(to_f32(r.integers(0, lattice, size=(n, d))))
    else:
        X = f32_to_bf16_bits(to_f32(r.standard_normal((m, d)) / np.sqrt(d)))
        Y = f32_to_bf16_bits(to_f32(r.standard_normal((n, d)) / np.sqrt(d)))
    if masses == "uniform":
        a, b = uniform_masses(m), uniform_masses(n)
    elif masses == "dirichlet":
        a, b = dirichlet_masses(r, m), dirichlet_masses(r, n)
    else:
        a, b = zipf_masses(r, m), zipf_masses(r, n)
    return X.reshape(m, d), a, Y.reshape(n, d), b


def _stroke_image(r, side: int) -> np.ndarray:
    """8-bit intensities of 1..3 thick random strokes (quadratic curves) on a
    dark background, blurred one pixel: most pixels are exactly 0."""
    img = np.zeros((side, side))
    yy, xx = np.mgrid[0:side, 0:side].astype(np.float64)
    for _ in range(int(r.integers(1, 4))):
        p0, p1, p2 = r.uniform(0.15 * side, 0.85 * side, size=(3, 2))
        width = r.uniform(0.9, 1.8)
        for t in np.linspace(0.0, 1.0, 4 * side):
            c = (1 - t) ** 2 * p0 + 2 * (1 - t) * t * p1 + t ** 2 * p2
            img = np.maximum(img, np.exp(-((yy - c[0]) ** 2 + (xx - c[1]) ** 2) / (2 * width ** 2)))
    q = np.floor(255.0 * img + 0.5)
    q[q < 24] = 0.0  # background
    return q


def _smooth_image(r, side: int) -> np.ndarray:
    """8-bit intensities of a smooth positive density: 2..6 Gaussian bumps of
    random width and weight plus a floor, so every pixel has mass."""
    yy, xx = np.mgrid[0:side, 0:side].astype(np.float64)
    img = np.full((side, side), 0.05)
    for _ in range(int(r.integers(2, 7))):
        cy, cx = r.uniform(0, side, size=2)
        w = r.uniform(0.05, 0.3) * side
        img += r.uniform(0.2, 1.0) * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * w ** 2))
    return np.floor(1.0 + 254.0 * img / img.max() + 0.5)


def lattice_hist_2d(num_images: int = 1024, side: int = 32, style: str = "smooth",
                    seed: int = SEEDS["lattice_hist_2d"]) -> PairSet:
    """Pixel-grid histograms: image k (stream k of the seed) on a side x side
    grid; points are the integer (row, col) of every pixel (FP32, exact), the
    masses the 8-bit intensities normalised in FP64 then rounded to FP32;
    pair p compares image p (suppliers) with image (p + 1) mod N."""
    yy, xx = np.mgrid[0:side, 0:side]
    grid = to_f32(np.stack([yy.ravel(), xx.ravel()], 1))
    sets = []
    for k in range(num_images):
        r = rng_for(seed + (0 if style == "smooth" else 100), k)
        img = _smooth_image(r, side) if style == "smooth" else _stroke_image(r, side)
        w = img.ravel().astype(np.float64)
        sets.append((grid, to_f32(w / w.sum())))
    Xc, ac, xo = _concat(sets, 2)
    pair_x = np.arange(num_images, dtype=np.int32)
    pair_y = ((np.arange(num_images) + 1) % num_images).astype(np.int32)
    return PairSet("lattice_hist_2d", 2, Xc, ac, xo, Xc, ac, xo, pair_x=pair_x, pair_y=pair_y, metric="l2",
                   meta={"num_images": num_images, "side": side, "style": style, "seed": seed})


def colour_image(k: int, height: int = 256, width: int = 256, seed: int = SEEDS["colour_images"]) -> np.ndarray:
    """Seeded smooth RGB image (uint8, height x width x 3): each channel a sum
    of a few random low-frequency waves and bumps, scaled to 0..255."""
    r = rng_for(seed, k)
    yy, xx = np.mgrid[0:height, 0:width].astype(np.float64)
    yy /= height
    xx /= width
    out = np.zeros((height, width, 3))
    for c in range(3):
        f = np.zeros((height, width))
        for _ in range(3):
            fy, fx, ph = r.uniform(0.5, 3.0), r.uniform(0.5, 3.0), r.uniform(0, 2 * np.pi)
            f += r.uniform(0.3, 1.0) * np.sin(2 * np.pi * (fy * yy + fx * xx) + ph)
        for _ in range(2):
            cy, cx, w = r.uniform(0, 1), r.uniform(0, 1), r.uniform(0.05, 0.3)
            f += r.uniform(-1.0, 1.0) * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * w ** 2))
        f = (f - f.min()) / max(f.max() - f.min(), 1e-12)
        out[..., c] = f * r.uniform(0.6, 1.0) + r.uniform(0.0, 0.3)
    return np.clip(np.floor(255.0 * out / max(out.max(), 1e-12) + 0.5), 0, 255).astype(np.uint8)
