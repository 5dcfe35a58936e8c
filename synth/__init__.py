"""Seeded synthetic inputs for the star-M truncated tensor SVD workloads.

This module only *builds inputs*: tensors, transform matrices and the
parameters each workload names.  It holds none of the method's arithmetic
(no mode-3 products, no SVDs, no rank selection), so both the FP64 oracle
and the GPU path can consume what it returns without sharing any code.

Layout convention (Section 3 of the paper: all data column-major).  A tensor
of shape m x p x n is returned as a NumPy array of shape (m, p, n) in Fortran
order, i.e. element (a, b, i) sits at flat offset a + b*m + i*m*p and every
frontal slice A[:, :, i] is one contiguous m x p column-major matrix.

The real datasets of the paper (climate reanalysis, Taylor-Green vortex CFD,
X-ray diffuse scattering) are not available; the generators below produce
inputs with the same shapes and comparable structure (smooth separable
fields plus noise, power-law random fields, low-rank plus noise).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "dct2_matrix",
    "haar_orthogonal",
    "skew_parameter",
    "planted_lowrank",
    "climate_like",
    "turbulence_like",
    "cp_lowrank",
    "ragged_batch",
    "Workload",
    "workload",
]


# ---------------------------------------------------------------------------
# transform matrices
# ---------------------------------------------------------------------------

def dct2_matrix(n: int) -> np.ndarray:
    """Orthonormal DCT-II matrix, n x n, FP64.

    Row i is the i-th cosine basis vector, so applying it along mode 3 maps
    tube position j to frequency i:  M[i, j] = sqrt(2/n) * lam_i *
    cos(pi * i * (2j + 1) / (2n)) with lam_0 = 1/sqrt(2), lam_i = 1 otherwise.
    The paper names the DCT as its transform (Section 2.2, "Choice of M") but
    does not print a normalisation; the orthonormal one is the choice that
    keeps the Eckart-Young guarantee of Section 2.3.
    """
    i = np.arange(n, dtype=np.float64)[:, None]
    j = np.arange(n, dtype=np.float64)[None, :]
    M = np.sqrt(2.0 / n) * np.cos(np.pi * i * (2.0 * j + 1.0) / (2.0 * n))
    M[0, :] *= 1.0 / np.sqrt(2.0)
    return np.ascontiguousarray(M)


def haar_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    """Random orthogonal n x n matrix: QR of a seeded Gaussian, with the sign
    of each column of Q fixed by the sign of R's diagonal (Haar distributed,
    deterministic for a given generator state)."""
    G = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(G)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return np.ascontiguousarray(Q * d[None, :])


def skew_parameter(n: int, rng: np.random.Generator, scale: float = 0.5) -> np.ndarray:
    """Skew-symmetric parameter K0 = scale * (W - W^T) / sqrt(n), W ~ N(0,1).

    The transform of the differentiation workload is the Cayley map of this
    parameter; the map itself is applied by the consumer, not here."""
    W = rng.standard_normal((n, n))
    return np.ascontiguousarray(scale * (W - W.T) / np.sqrt(n))


# ---------------------------------------------------------------------------
# tensors
# ---------------------------------------------------------------------------

def _fortran(x: np.ndarray, dtype) -> np.ndarray:
    return np.asfortranarray(x, dtype=dtype)


def planted_lowrank(m: int, p: int, n: int, rank: int, scale: float,
                    rng: np.random.Generator, dtype=np.float64) -> np.ndarray:
    """N(0,1) entries plus `scale` times a sum of `rank` outer products
    a_l o b_l o c_l of unnormalised Gaussian vectors."""
    A = rng.standard_normal((m, p, n))
    for _ in range(rank):
        a = rng.standard_normal(m)
        b = rng.standard_normal(p)
        c = rng.standard_normal(n)
        A += scale * np.einsum("a,b,c->abc", a, b, c)
    return _fortran(A, dtype)


def cp_lowrank(m: int, p: int, n: int, rank: int, noise: float,
               rng: np.random.Generator, dtype=np.float32) -> np.ndarray:
    """Sum of `rank` Gaussian outer products, scaled to unit RMS, plus
    N(0, noise^2) entries.  Built slice by slice in FP64 then cast."""
    a = rng.standard_normal((m, rank))
    b = rng.standard_normal((p, rank))
    c = rng.standard_normal((n, rank))
    # RMS of the low-rank part, computed from the factor Gram matrices
    gram = (a.T @ a) * (b.T @ b) * (c.T @ c)
    rms = math.sqrt(max(gram.sum(), 1e-300) / (m * p * n))
    A = np.empty((m, p, n), dtype=dtype, order="F")
    ab = [np.ascontiguousarray(a * c[i][None, :]) for i in range(n)]
    for i in range(n):
        sl = (ab[i] @ b.T) / rms
        if noise > 0:
            sl = sl + noise * rng.standard_normal((m, p))
        A[:, :, i] = sl
    return A


def climate_like(m: int = 512, p: int = 1024, n: int = 256, terms: int = 40,
                 noise: float = 0.01, rng: np.random.Generator | None = None,
                 dtype=np.float32) -> np.ndarray:
    """Smooth lat x lon x time field from `terms` separable sinusoids plus
    `noise` * RMS Gaussian noise.

    Term l is a_l * cos(theta)^|m_l| * cos(j_l theta + g_l) * cos(m_l phi + al_l)
    * cos(2 pi t / T_l + b_l) with theta the latitude in [-pi/2, pi/2], phi
    the longitude in [0, 2 pi), t the time index in steps of 6 h and T_l
    either 4 steps (diurnal) or 1460 steps (annual), each with probability 1/2;
    m_l ~ U{0..12}, j_l ~ U{0..8}, a_l = 1 / (1 + m_l + j_l), phases U[0, 2pi).
    It stands in for the climate reanalysis tensor of Section 4.1.
    """
    rng = np.random.default_rng(2) if rng is None else rng
    theta = np.linspace(-np.pi / 2, np.pi / 2, m)
    phi = np.arange(p) * (2 * np.pi / p)
    t = np.arange(n, dtype=np.float64)
    F_lat = np.empty((m, terms))
    F_lon = np.empty((p, terms))
    F_t = np.empty((n, terms))
    for l in range(terms):
        ml = int(rng.integers(0, 13))
        jl = int(rng.integers(0, 9))
        T = 4.0 if rng.random() < 0.5 else 1460.0
        g, al, be = rng.uniform(0, 2 * np.pi, 3)
        amp = 1.0 / (1.0 + ml + jl)
        F_lat[:, l] = amp * np.cos(theta) ** ml * np.cos(jl * theta + g)
        F_lon[:, l] = np.cos(ml * phi + al)
        F_t[:, l] = np.cos(2 * np.pi * t / T + be)
    # RMS of the smooth part from the factor Grams
    gram = (F_lat.T @ F_lat) * (F_lon.T @ F_lon) * (F_t.T @ F_t)
    rms = math.sqrt(max(gram.sum(), 1e-300) / (m * p * n))
    A = np.empty((m, p, n), dtype=dtype, order="F")
    sigma = noise * rms
    for i in range(n):
        sl = (F_lat * F_t[i][None, :]) @ F_lon.T
        if sigma > 0:
            sl = sl + sigma * rng.standard_normal((m, p))
        A[:, :, i] = sl
    return A


def climate6_like(lat: int = 73, lon: int = 144, levels: int = 17, days: int = 365,
                  years: int = 2, terms: int = 40, noise: float = 0.01,
                  rng: np.random.Generator | None = None, dtype=np.float32) -> np.ndarray:
    """Order-6 climate-like field lat x lon x level x time-of-day (4) x
    day-of-year x year, the layout of the paper's 6-way reanalysis tensor
    (Section 4.1: the 6-hourly time axis split into time of day, day and
    year).  Term l is a_l * cos(theta)^|m_l| cos(j_l theta + g_l)
    * cos(m_l phi + al_l) * cos(pi k_l z + d_l) * cos(2 pi t / T_l + b_l), with z
    the level in [0, 1], k_l ~ U{0..3}, t = tod + 4 (day + days * year) the
    6-hourly time index and T_l in {4, 1460} steps as in climate_like; plus
    `noise` * RMS Gaussian noise.  Column-major (Fortran) order."""
    rng = np.random.default_rng(12) if rng is None else rng
    nt = 4 * days * years
    theta = np.linspace(-np.pi / 2, np.pi / 2, lat)
    phi = np.arange(lon) * (2 * np.pi / lon)
    z = np.linspace(0.0, 1.0, levels) if levels > 1 else np.zeros(1)
    t = np.arange(nt, dtype=np.float64)
    F_lat = np.empty((lat, terms))
    F_lon = np.empty((lon, terms))
    F_lev = np.empty((levels, terms))
    F_t = np.empty((nt, terms))
    for l in range(terms):
        ml = int(rng.integers(0, 13))
        jl = int(rng.integers(0, 9))
        kl = int(rng.integers(0, 4))
        T = 4.0 if rng.random() < 0.5 else 1460.0
        g, al, dl, be = rng.uniform(0, 2 * np.pi, 4)
        amp = 1.0 / (1.0 + ml + jl)
        F_lat[:, l] = amp * np.cos(theta) ** ml * np.cos(jl * theta + g)
        F_lon[:, l] = np.cos(ml * phi + al)
        F_lev[:, l] = np.cos(np.pi * kl * z + dl)
        F_t[:, l] = np.cos(2 * np.pi * t / T + be)
    # (lat lon) x terms Khatri-Rao factor and (level time) x terms coefficients
    KR = (F_lat[:, None, :] * F_lon[None, :, :]).reshape(lat * lon, terms, order="F")
    N = levels * nt
    gram = (F_lat.T @ F_lat) * (F_lon.T @ F_lon) * (F_lev.T @ F_lev) * (F_t.T @ F_t)
    rms = math.sqrt(max(gram.sum(), 1e-300) / (lat * lon * N))
    sigma = noise * rms
    A = np.empty((lat * lon, N), dtype=dtype, order="F")
    chunk = max(1, (1 << 24) // (lat * lon))
    for s0 in range(0, N, chunk):
        s1 = min(N, s0 + chunk)
        idx = np.arange(s0, s1)
        C = F_lev[idx % levels] * F_t[idx // levels]          # (s1-s0) x terms
        block = KR @ C.T
        if sigma > 0:
            block += sigma * rng.standard_normal(block.shape)
        A[:, s0:s1] = block
    return A.reshape((lat, lon, levels, 4, days, years), order="F")


def turbulence_like(m: int = 2048, p: int = 1024, n: int = 256,
                    rng: np.random.Generator | None = None,
                    dtype=np.float32, workers: int = -1) -> np.ndarray:
    """3-D Gaussian random field with a k^(-5/3) energy spectrum.

    White Gaussian noise is filtered in Fourier space by |k|^(-11/6) (the
    amplitude that gives E(k) ~ k^(-5/3) in three dimensions), the k = 0 mode
    is removed and the field is normalised to unit variance.  The last mode
    (n) plays the role of time snapshots.  It stands in for the turbulent
    CFD tensor of Section 4.2.
    """
    import scipy.fft as sfft

    rng = np.random.default_rng(4) if rng is None else rng
    # generate in C order (n, p, m) so the Fortran (m, p, n) view is free
    w = rng.standard_normal((n, p, m), dtype=np.float32)
    W = sfft.rfftn(w, workers=workers)
    del w
    kn = np.fft.fftfreq(n).astype(np.float32)[:, None, None]
    kp = np.fft.fftfreq(p).astype(np.float32)[None, :, None]
    km = np.fft.rfftfreq(m).astype(np.float32)[None, None, :]
    for i in range(n):
        k2 = kn[i] ** 2 + kp ** 2 + km ** 2
        k2 = k2[0]
        with np.errstate(divide="ignore"):
            filt = np.where(k2 > 0, k2 ** (-11.0 / 12.0), 0.0).astype(np.float32)
        W[i] *= filt
    f = sfft.irfftn(W, s=(n, p, m), workers=workers)
    del W
    f = f.astype(dtype, copy=False)
    f -= f.mean(dtype=np.float64)
    f /= np.float32(f.std(dtype=np.float64))
    return f.transpose(2, 1, 0)  # (m, p, n) Fortran-ordered view


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    """One named input: tensor(s), transform(s) and truncation parameters."""
    name: str
    A: object                      # ndarray (m, p, n) or list of them
    M: object                      # ndarray (n, n) or list of them
    mode: object                   # "I" / "II" or list
    k: object = None               # t-SVDM-I rank (or list)
    eps: object = None             # t-SVDM-II tolerance (or list)
    extra: dict = field(default_factory=dict)


def ragged_batch(count: int = 512, seed: int = 3, lo: int = 32, hi: int = 384,
                 nlo: int = 8, nhi: int = 96, dtype=np.float32,
                 size_scale: float = 1.0) -> Workload:
    """Many independent tensors of uneven shape (the batching workload).

    Tensor t uses its own generator spawned from SeedSequence(seed); m, p are
    uniform in [lo, hi], n uniform in [nlo, nhi], the CP rank uniform in
    [2, 32], noise 1e-2; M is a Haar orthogonal matrix; even t use t-SVDM-I
    with k = 16 and odd t use t-SVDM-II with tolerance 1e-2.  `size_scale`
    shrinks m, p, n proportionally for quick tests.
    """
    children = np.random.SeedSequence(seed).spawn(count)
    As, Ms, modes, ks, epss = [], [], [], [], []
    for t, ss in enumerate(children):
        rng = np.random.default_rng(ss)
        m = int(rng.integers(lo, hi + 1))
        p = int(rng.integers(lo, hi + 1))
        n = int(rng.integers(nlo, nhi + 1))
        R = int(rng.integers(2, 33))
        if size_scale != 1.0:
            m = max(4, int(round(m * size_scale)))
            p = max(4, int(round(p * size_scale)))
            n = max(2, int(round(n * size_scale)))
        As.append(cp_lowrank(m, p, n, R, 1e-2, rng, dtype=dtype))
        Ms.append(haar_orthogonal(n, rng))
        if t % 2 == 0:
            modes.append("I"); ks.append(16); epss.append(None)
        else:
            modes.append("II"); ks.append(None); epss.append(1e-2)
    return Workload("ragged_batch", As, Ms, modes, ks, epss)


def workload(name: str, small: bool = False) -> Workload:
    """The five named workloads.

    planted     : 64x48x16, N(0,1) + rank-4 planted part (scale 10), DCT-II,
                  t-SVDM-I k=8, FP64.
    climate     : 512x1024x256 climate-like field, DCT-II, t-SVDM-II tol 1e-3.
    ragged      : 512 uneven tensors (see ragged_batch).
    turbulence  : 2048x1024x256 k^-5/3 random field, Haar M, t-SVDM-II tol 1e-2.
    cayley      : 256x256x64 CP rank-24 + 5% noise, k=16, M = Cayley(K0).
    climate6    : 73x144x17x4x365x2 order-6 climate-like field, DCT-II along
                  every mode >= 3 (M is a list), t-SVDM-II tol 1e-2.

    `small=True` returns the same recipe at reduced size for quick tests.
    """
    if name == "planted":
        rng = np.random.default_rng(1)
        A = planted_lowrank(64, 48, 16, 4, 10.0, rng)
        return Workload(name, A, dct2_matrix(16), "I", k=8)
    if name == "climate":
        m, p, n = (96, 160, 32) if small else (512, 1024, 256)
        A = climate_like(m, p, n, rng=np.random.default_rng(2))
        return Workload(name, A, dct2_matrix(n), "II", eps=1e-3)
    if name == "ragged":
        return ragged_batch(count=24 if small else 512,
                            size_scale=0.35 if small else 1.0)
    if name == "climate6":
        dims = (24, 36, 5, 4, 12, 2) if small else (73, 144, 17, 4, 365, 2)
        A = climate6_like(*dims[:3], days=dims[4], years=dims[5], rng=np.random.default_rng(12))
        return Workload(name, A, [dct2_matrix(n) for n in dims[2:]], "II", eps=1e-2)
    if name == "turbulence":
        m, p, n = (192, 128, 32) if small else (2048, 1024, 256)
        rng = np.random.default_rng(4)
        A = turbulence_like(m, p, n, rng=rng)
        M = haar_orthogonal(n, np.random.default_rng(40))
        return Workload(name, A, M, "II", eps=1e-2)
    if name == "cayley":
        m, p, n = (48, 40, 12) if small else (256, 256, 64)
        rng = np.random.default_rng(5)
        A = cp_lowrank(m, p, n, 24 if not small else 6, 0.05, rng, dtype=np.float32)
        K0 = skew_parameter(n, np.random.default_rng(50))
        return Workload(name, A, None, "I", k=16 if not small else 4,
                        extra={"K0": K0})
    raise KeyError(name)
