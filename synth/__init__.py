"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and lays out input arrays.  It holds
none of the deblurring arithmetic (no wavelet transform, no blur, no sparse
operator algebra), so that the CPU oracle and the GPU library can both be fed
from it without sharing any step of the method.

Everything is drawn with numpy's PCG64 (``numpy.random.default_rng``) in
float64.  The paper's test images (Sec. 5, the 1024x1024 "book" and "confocal"
pictures) are not available; the piecewise-smooth generator below stands in
for them with values in [0, 1], the range the paper rescales its images to
(Sec. 5).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict

import numpy as np

__all__ = [
    "piecewise_image", "noise", "psf_isotropic", "psf_rotating", "PsfField",
    "power_start", "banded_operator", "local_operator", "Workload", "WORKLOADS", "batched_problems",
]


def piecewise_image(n: int, seed: int) -> np.ndarray:
    """n x n float64 image in [0, 1]: a linear ramp with 8 painted shapes.

    Draw order (fixed, so the image is a function of ``seed`` only):
    background c0 ~ U[0, .5], c1, c2 ~ U[-.25, .25] giving
    c0 + c1*col/n + c2*row/n; then 8 shapes, each a disk (probability 1/2:
    centre ~ U over the image, radius ~ U[n/16, n/4]) or an axis-aligned
    rectangle (two corners ~ U over the image), filled with its own intensity
    ~ U[0, 1] and overwriting what is below; finally clipped to [0, 1].
    """
    rng = np.random.default_rng(seed)
    row, col = np.meshgrid(np.arange(n, dtype=np.float64),
                           np.arange(n, dtype=np.float64), indexing="ij")
    c0 = rng.uniform(0.0, 0.5)
    c1 = rng.uniform(-0.25, 0.25)
    c2 = rng.uniform(-0.25, 0.25)
    img = c0 + c1 * col / n + c2 * row / n
    for _ in range(8):
        if rng.random() < 0.5:
            cy, cx = rng.uniform(0.0, n, size=2)
            rad = rng.uniform(n / 16.0, n / 4.0)
            mask = (row - cy) ** 2 + (col - cx) ** 2 <= rad * rad
        else:
            ys = np.sort(rng.uniform(0.0, n, size=2))
            xs = np.sort(rng.uniform(0.0, n, size=2))
            mask = (row >= ys[0]) & (row <= ys[1]) & (col >= xs[0]) & (col <= xs[1])
        img[mask] = rng.uniform(0.0, 1.0)
    return np.clip(img, 0.0, 1.0)


def noise(n: int, sigma: float, seed: int) -> np.ndarray:
    """White Gaussian noise b ~ N(0, sigma^2 I) on an n x n grid (Sec. 1.1)."""
    return np.random.default_rng(seed).normal(0.0, sigma, size=(n, n))


@dataclass
class PsfField:
    """Per-source-pixel Gaussian PSF parameters, row-major (row, col) arrays.

    ``sig_major``/``sig_minor`` are the standard deviations (pixels) along the
    principal axes; ``angle`` (radians) turns the major axis from the column
    (x) axis toward the row (y) axis.  ``trunc`` is the Mahalanobis radius at
    which each PSF is cut off.
    """
    n: int
    sig_major: np.ndarray
    sig_minor: np.ndarray
    angle: np.ndarray
    trunc: float = 3.0

    @property
    def radius(self) -> int:
        """Largest integer offset any truncated PSF of the field can reach."""
        return int(math.floor(self.trunc * float(max(self.sig_major.max(), self.sig_minor.max()))))


def psf_isotropic(n: int, s0: float = 1.0, s1: float = 3.0, trunc: float = 3.0) -> PsfField:
    """Isotropic field sigma(col) = s0 + (s1 - s0) * col / n (constant down columns)."""
    col = np.arange(n, dtype=np.float64)[None, :].repeat(n, axis=0)
    sig = s0 + (s1 - s0) * col / n
    return PsfField(n, sig.copy(), sig.copy(), np.zeros((n, n)), trunc)


def psf_rotating(n: int, major: float, minor: float, trunc: float = 3.0) -> PsfField:
    """Anisotropic field with fixed axis lengths whose angle is pi * col / n."""
    col = np.arange(n, dtype=np.float64)[None, :].repeat(n, axis=0)
    return PsfField(n, np.full((n, n), float(major)), np.full((n, n), float(minor)),
                    math.pi * col / n, trunc)


def psf_stationary(n: int, major: float, minor: float, angle: float = 0.0, trunc: float = 3.0) -> PsfField:
    """The same Gaussian PSF at every pixel: H is a circular convolution."""
    return PsfField(n, np.full((n, n), float(major)), np.full((n, n), float(minor)),
                    np.full((n, n), float(angle)), trunc)


def power_start(size: int, seed: int) -> np.ndarray:
    """Seeded N(0, 1) start vector for the power iteration."""
    return np.random.default_rng(seed).standard_normal(size)


def banded_operator(size: int, nnz_per_row: float, seed: int, far_fraction: float = 0.1,
                    band: int = 64):
    """A seeded random sparse square matrix (CSR, float64) with a dominant
    diagonal, a band of near entries and a few far entries per row.

    It mimics the storage-relevant structure of a thresholded wavelet-domain
    operator (strong diagonal, entries concentrated near it, uneven row
    lengths) so that full-size kernel parity can run on inputs the oracle did
    not have to build.  Returns (rowptr int64, col int32, val float64).
    """
    rng = np.random.default_rng(seed)
    lens = rng.geometric(1.0 / max(nnz_per_row - 1.0, 1.0), size=size)
    lens = np.minimum(lens, 8 * int(nnz_per_row) + 1)
    rows = np.repeat(np.arange(size, dtype=np.int64), lens)
    m = rows.size
    far = rng.random(m) < far_fraction
    off = rng.integers(-band, band + 1, size=m)
    offf = rng.integers(0, size, size=m)
    cols = np.where(far, offf, (rows + off) % size)
    key = np.unique(np.concatenate([rows * size + cols,
                                    np.arange(size, dtype=np.int64) * (size + 1)]))
    r = key // size
    c = (key % size).astype(np.int32)
    val = rng.normal(0.0, 0.3 / math.sqrt(nnz_per_row), size=key.size)
    diag = r == c
    val[diag] = rng.uniform(0.4, 1.0, size=int(diag.sum()))
    rowptr = np.zeros(size + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr, c, val


def _bands(n: int, levels: int):
    """(level, orientation, side, first index) of each subband in canonical
    order: the coarsest approximation, then per level J..1 the three details."""
    out = [(levels, 3, n >> levels, 0)]
    for lev in range(levels, 0, -1):
        sd = n >> lev
        for o in range(3):
            out.append((lev, o, sd, (o + 1) * sd * sd))
    return out


def local_operator(n: int, levels: int, nnz_per_px: float, seed: int, radius: int = 3, coarse_from: int = 0,
                   far: int = 0):
    """A seeded sparse N x N matrix (N = n^2, rows and columns in canonical
    subband order) with the storage-relevant structure of a thresholded
    wavelet-domain operator of a slowly varying blur, at full size.

    Row a (subband of level la, position (i, j)) keeps entries in the subbands
    of levels la - 1 .. la + 1 at displacements |di|, |dj| <= radius around
    (i, j) scaled to the column subband's side, with magnitude
    amp * exp(-(di^2 + dj^2) / (2 w^2)): amp = 2^-|level gap| (times 0.35
    across orientations) and a width w that grows smoothly from 0.7 to 2.3
    across the image columns.  The largest of these are kept (ties in a seeded
    random order), as many as make nnz_per_px * n^2 entries in all with the
    additions below (fewer only where wrapping on a small subband repeats an
    entry); each kept value gets a random sign and 5 % multiplicative noise.

    With ``coarse_from`` > 0, every row of a detail subband of level
    >= coarse_from also keeps, like the long rows of a coarse atom that
    overlaps many finer ones, entries in the same orientation two levels finer
    at every displacement in [-8, 8]^2 and three levels finer on the lattice
    {-24, -18, ..., 24}^2 (magnitude just above the smallest kept one).
    ``far`` extra entries (that magnitude) join rows of the finest level: half at a level gap of 4
    (when the transform has 5 levels or more), the others at a displacement of
    129..200 positions in a column subband of side >= 512, beyond any short
    band-relative code.  Returns (rowptr int64, col int32, val float64).
    """
    rng = np.random.default_rng(seed)
    N = n * n
    bands = _bands(n, levels)
    offs = np.arange(-radius, radius + 1)
    DI, DJ = (a.ravel() for a in np.meshgrid(offs, offs, indexing="ij"))
    d2 = (DI * DI + DJ * DJ).astype(np.float64)
    pairs = [(A, B, 0.5 ** abs(A[0] - B[0]) * (1.0 if A[1] == B[1] else 0.35))
             for A in bands for B in bands if abs(A[0] - B[0]) <= 1]

    def width(A):
        sa = A[2]
        j = np.arange(sa * sa) % sa
        return 0.7 + 1.6 * (j + 0.5) / sa

    widths = {A[3]: width(A) for A in bands}
    d2v, d2c = np.unique(d2, return_counts=True)

    cum = np.concatenate([[0], np.cumsum(d2c)])   # entries with d2 below the k-th distinct value

    def count(tau):
        tot = 0
        for A, B, amp in pairs:
            if amp > tau:   # kept iff d2 < 2 w^2 ln(amp / tau)
                lim = 2.0 * widths[A[3]] ** 2 * math.log(amp / tau)
                tot += int(cum[np.searchsorted(d2v, lim, side="left")].sum())
        return tot

    # the coarse rows' long runs of finer columns (added below, outside the threshold)
    runs = []
    if coarse_from > 0:
        o2 = np.arange(-8, 9)
        o3 = np.arange(-24, 25, 6)
        for A in bands:
            la, oa, sa, fa = A
            if oa == 3 or la < coarse_from:
                continue
            for g, oo in ((2, o2), (3, o3)):
                B = [b for b in bands if b[0] == la - g and b[1] == oa]
                if B:
                    runs.append((A, B[0], oo))
    far_rows, far_cols = [], []
    if far:
        fine = [B for B in bands if B[0] == 1]
        for t in range(far):
            A = fine[t % 3]
            a = A[3] + int(rng.integers(0, A[2] * A[2]))
            if t % 2 == 0 and levels >= 5:   # level gap 4: a coarse column
                B = [b for b in bands if b[0] == 5][t % 3]
                far_cols.append(B[3] + int(rng.integers(0, B[2] * B[2])))
            else:
                B = fine[(t // 2) % 3]
                if B[2] < 512:
                    continue
                i, j = divmod(a - A[3], A[2])
                d = int(rng.integers(129, 201)) * (1 if rng.random() < 0.5 else -1)
                far_cols.append(B[3] + ((i + d) % B[2]) * B[2] + j)
            far_rows.append(a)
    extra = sum(A[2] * A[2] * oo.size ** 2 for A, B, oo in runs) + len(far_rows)
    target = nnz_per_px * N - extra
    lo, hi = 1e-12, 1.0
    for _ in range(60):
        mid = math.sqrt(lo * hi)
        if count(mid) > target:
            lo = mid
        else:
            hi = mid
    tau = lo   # count(lo) > target: generate above lo, then keep the target's largest
    rows, cols, mags = [], [], []
    for A, B, amp in pairs:
        if amp <= tau:
            continue
        (la, oa, sa, fa), (lb, ob, sb, fb) = A, B
        i, j = np.divmod(np.arange(sa * sa), sa)
        ci, cj = (i * sb) // sa, (j * sb) // sa
        mag = amp * np.exp(-d2[None, :] / (2.0 * widths[fa][:, None] ** 2))
        keep = d2[None, :] < (2.0 * widths[fa] ** 2 * math.log(amp / tau))[:, None]   # as count() decides
        rr, kk = np.nonzero(keep)
        rows.append(fa + rr)
        cols.append(fb + ((ci[rr] + DI[kk]) % sb) * sb + (cj[rr] + DJ[kk]) % sb)
        mags.append(mag[rr, kk])
    if rows:   # the base entries: the `target` largest magnitudes (ties in a seeded random order)
        r0, c0, m0 = np.concatenate(rows), np.concatenate(cols), np.concatenate(mags)
        t = max(min(int(target), m0.size), 0)
        key = m0 * (1.0 + 1e-9 * rng.random(m0.size))   # seeded tie-break; selection only
        keep = np.sort(np.argpartition(-key, t - 1)[:t]) if 0 < t < m0.size else np.arange(t)
        rows, cols, mags = [r0[keep]], [c0[keep]], [m0[keep]]
    floor = float(np.min(mags[0])) if rows and mags[0].size else 1.0   # smallest kept base magnitude
    for A, B, oo in runs:
        (la, oa, sa, fa), (lb, ob, sb, fb) = A, B
        EI, EJ = (a.ravel() for a in np.meshgrid(oo, oo, indexing="ij"))
        i, j = np.divmod(np.arange(sa * sa), sa)
        ci, cj = (i * sb) // sa, (j * sb) // sa
        rows.append(np.repeat(fa + np.arange(sa * sa), EI.size))
        cols.append(fb + ((np.repeat(ci, EI.size) + np.tile(EI, sa * sa)) % sb) * sb
                    + (np.repeat(cj, EI.size) + np.tile(EJ, sa * sa)) % sb)
        mags.append(np.full(sa * sa * EI.size, 1.2 * floor))
    rows.append(np.array(far_rows, dtype=np.int64))
    cols.append(np.array(far_cols, dtype=np.int64))
    mags.append(np.full(len(far_rows), floor))
    r = np.concatenate(rows).astype(np.int64)
    c = np.concatenate(cols).astype(np.int64)
    m = np.concatenate(mags)
    key, first = np.unique(r * N + c, return_index=True)   # sorted by (row, col); wrap duplicates dropped
    m = m[first]
    val = m * np.where(rng.random(m.size) < 0.5, -1.0, 1.0) * (1.0 + 0.05 * rng.standard_normal(m.size))
    r = key // N
    rowptr = np.zeros(N + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    return np.cumsum(rowptr), (key % N).astype(np.int32), val


@dataclass
class Workload:
    """One named synthetic workload: image, blur field, basis and solver settings."""
    name: str
    n: int
    wavelet: str            # "haar" or "db4"
    levels: int
    nnz_per_px: int
    lam: float
    noise_sigma: float
    image_seed: int
    noise_seed: int
    power_seed: int
    iters: int
    field: str              # "isotropic" or "rotating"
    field_args: Dict[str, float] = field(default_factory=dict)
    tol: float = 1e-4       # float64 relative duality gap that ends a solve

    @property
    def nnz(self) -> int:
        return self.nnz_per_px * self.n * self.n

    def psf(self) -> PsfField:
        if self.field == "isotropic":
            return psf_isotropic(self.n, **self.field_args)
        return psf_rotating(self.n, **self.field_args)

    def image(self) -> np.ndarray:
        return piecewise_image(self.n, self.image_seed)

    def noise(self) -> np.ndarray:
        return noise(self.n, self.noise_sigma, self.noise_seed)


WORKLOADS: Dict[str, Workload] = {
    # 64^2 parity case: Haar, 3 levels, sigma = 1 + 2 col/n, 40 nnz/px, 200 iterations.
    "parity64": Workload("parity64", 64, "haar", 3, 40, 2e-3, 0.01, 1, 2, 3, 200,
                         "isotropic", {"s0": 1.0, "s1": 3.0}),
    # 512^2 precision case: db4, 5 levels, rotating 4/1 field, 30 nnz/px, 500 iterations.
    "precision512": Workload("precision512", 512, "db4", 5, 30, 1e-3, 0.01, 11, 12, 13, 500,
                             "rotating", {"major": 4.0, "minor": 1.0}),
    # 1024^2 case: db4, 6 levels, rotating 6/1 field, 20 nnz/px, gap-checked stop.
    "scale1024": Workload("scale1024", 1024, "db4", 6, 20, 5e-4, 0.005, 21, 22, 23, 2000,
                          "rotating", {"major": 6.0, "minor": 1.0}),
    # 256^2 warm-start case: db4, 4 levels, sigma = 1 + 2 col/n, 30 nnz/px.
    "learned256": Workload("learned256", 256, "db4", 4, 30, 1e-3, 0.01, 50000, 150000, 53, 500,
                           "isotropic", {"s0": 1.0, "s1": 3.0}, 1e-6),
}


def batched_problems(seed: int = 41, groups: int = 8, rhs: int = 8):
    """Draw the uneven batched case: ``groups`` operators, each shared by ``rhs``
    right-hand sides.  Per group: n ~ U{128, 256, 512, 1024}, levels = log2(n) - 4,
    nnz/px ~ U{20..40}, a PSF field (isotropic ramp a..b with a, b ~ U[1, 5], or
    rotating with minor ~ U[1, 2.5], major ~ U[minor, 5], each with probability
    1/2) and per right-hand side lambda ~ logU[1e-4, 1e-2] plus image/noise seeds.
    """
    rng = np.random.default_rng(seed)
    out = []
    for g in range(groups):
        n = int(rng.choice([128, 256, 512, 1024]))
        levels = int(round(math.log2(n))) - 4
        nnz_px = int(rng.integers(20, 41))
        if rng.random() < 0.5:
            a, b = rng.uniform(1.0, 5.0, size=2)
            psf = ("isotropic", {"s0": float(a), "s1": float(b)})
        else:
            mn = rng.uniform(1.0, 2.5)
            mj = rng.uniform(mn, 5.0)
            psf = ("rotating", {"major": float(mj), "minor": float(mn)})
        lams = np.exp(rng.uniform(math.log(1e-4), math.log(1e-2), size=rhs))
        seeds = rng.integers(0, 2**31 - 1, size=(rhs, 2))
        out.append({"n": n, "levels": levels, "nnz_per_px": nnz_px, "field": psf,
                    "lams": lams.tolist(), "seeds": seeds.tolist()})
    return out
