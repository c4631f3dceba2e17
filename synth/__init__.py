"""Seeded synthetic inputs for the sparse-HRIR renderer.

This module only draws random numbers and lays them out: HRIR sets shaped
like a measured database (directions x ears x 200 taps at 44.1 kHz), source
signals (white and pink noise), job lists, and initial factors.  It holds
none of the rendering or factorization arithmetic; both the FP64 oracle and
the GPU path take its outputs as plain inputs.

The one convolution below is part of the *definition* of the synthetic HRIR
set (each HRIR is a shared resonance filter convolved with a sparse
non-negative reflection filter, the model of Eq. (1)); it is computed with
``numpy.convolve`` and is not shared with either implementation.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

FS = 44100.0          # HRIR sampling rate (Sec. IV-A: CD-quality data)
M_TAPS = 200          # HRIR length in taps (Sec. IV-C: M = 200)
HEAD_RADIUS_M = 0.096  # half of the 19.2 cm head diameter quoted in Sec. IV-C
SPEED_OF_SOUND = 343.0


# ---------------------------------------------------------------------------
# HRIR set
# ---------------------------------------------------------------------------
def resonance(rng: np.random.Generator, lf: int = 32, fs: float = FS) -> np.ndarray:
    """Resonance filter: sum of 3 exponentially damped sinusoids, unit L2 norm.

    Frequencies U(2, 8) kHz, decay constants U(0.2, 1) ms, phases U(0, 2pi).
    """
    n = np.arange(lf, dtype=np.float64)
    r = np.zeros(lf)
    for _ in range(3):
        fc = rng.uniform(2000.0, 8000.0)
        tau = rng.uniform(0.2e-3, 1.0e-3)
        phi = rng.uniform(0.0, 2.0 * math.pi)
        r += np.exp(-n / (fs * tau)) * np.cos(2.0 * math.pi * fc * n / fs + phi)
    return r / np.linalg.norm(r)


def directions(n_az: int, n_el: int) -> tuple[np.ndarray, np.ndarray]:
    """Interaural-polar grid: azimuths uniform in [-80, 80] deg, elevations
    from -45 deg in 5.625 deg steps.  Returns (az, el) in radians, flattened
    az-major (direction d = i_az * n_el + i_el)."""
    az = np.deg2rad(np.linspace(-80.0, 80.0, n_az)) if n_az > 1 else np.zeros(1)
    el = np.deg2rad(-45.0 + 5.625 * np.arange(n_el))
    AZ, EL = np.meshgrid(az, el, indexing="ij")
    return AZ.ravel(), EL.ravel()


def woodworth_itd(theta: np.ndarray) -> np.ndarray:
    """Spherical-head interaural time difference (a/c)(theta + sin theta)."""
    return HEAD_RADIUS_M / SPEED_OF_SOUND * (theta + np.sin(theta))


@dataclass
class HrirSet:
    r: np.ndarray        # f64[lf]      true resonance filter (unit norm)
    g: np.ndarray        # f64[F][lg]   true reflection filters, F = 2 * D (filter = 2*d + ear)
    h: np.ndarray        # f64[F][M]    HRIRs, h = r * g (full length lf + lg - 1 = M)
    az: np.ndarray       # f64[D] radians
    el: np.ndarray       # f64[D] radians
    onset: np.ndarray    # i64[F]
    contra: np.ndarray = None   # bool[F]: the ear on the far side of the head from the source

    @property
    def n_filters(self) -> int:
        return self.h.shape[0]


def hrir_set(seed: int, n_az: int, n_el: int, lf: int = 32, m: int = M_TAPS,
             n_pinna: int = 11, noise: float = 1e-3, shadow: float = 0.0) -> HrirSet:
    """Synthetic HRIR set: F = 2 * n_az * n_el filters of m taps.

    Reflection filter (length lg = m - lf + 1): a unit tap at the onset
    (0..40 samples, from the Woodworth ITD; the ear facing the source is
    earlier), ``n_pinna`` pinna taps 2..30 samples after the onset whose
    offsets move smoothly with elevation and whose gains decay geometrically
    (u_j * 0.8**j, u_j ~ U(0.1, 1)), plus non-negative noise U(0, noise) on
    every tap.  HRIR = resonance * reflection (full convolution, length m).

    shadow > 0 adds head shadow on the contralateral ear (the later onset):
    its HRIR is (resonance * lp) * reflection, truncated to m taps, with the
    low-pass lp_j = a^j / sum (j < 8), a = shadow |itd| / itd(90 deg), so the
    resonance of that ear differs with direction and from the ipsilateral one.
    """
    rng = np.random.default_rng(seed)
    lg = m - lf + 1
    r = resonance(rng, lf)
    az, el = directions(n_az, n_el)
    D = az.size
    base = [rng.uniform(2.0, 30.0, size=n_pinna) for _ in range(2)]
    psi = [rng.uniform(0.0, 2.0 * math.pi, size=n_pinna) for _ in range(2)]
    w90 = woodworth_itd(np.array(math.pi / 2.0))
    g = np.zeros((2 * D, lg))
    onset = np.zeros(2 * D, dtype=np.int64)
    contra = np.zeros(2 * D, dtype=bool)
    res_f = [r] * (2 * D)
    for d in range(D):
        itd = woodworth_itd(np.array(az[d])) / w90
        for e in range(2):
            f = 2 * d + e
            sign = -1.0 if e == 0 else 1.0
            on = int(round(20.0 + sign * 20.0 * float(itd)))
            on = min(max(on, 0), 40)
            contra[f] = sign * float(itd) > 0.0
            if shadow > 0.0 and contra[f]:
                a = shadow * abs(float(itd))
                lp = a ** np.arange(8)
                res_f[f] = np.convolve(r, lp / lp.sum())
            onset[f] = on
            g[f, on] += 1.0
            u = rng.uniform(0.1, 1.0, size=n_pinna)
            off = np.clip(np.round(base[e] + 4.0 * np.sin(el[d] + psi[e])), 2, 30).astype(np.int64)
            for j in range(n_pinna):
                g[f, on + off[j]] += u[j] * 0.8 ** (j + 1)
            g[f] += rng.uniform(0.0, noise, size=lg)
    h = np.stack([np.convolve(res_f[f], g[f])[:m] for f in range(2 * D)])
    return HrirSet(r=r, g=g, h=h, az=az, el=el, onset=onset, contra=contra)


# ---------------------------------------------------------------------------
# Source signals
# ---------------------------------------------------------------------------
def white(seed: int, n: int, sigma: float = 0.1) -> np.ndarray:
    """White Gaussian noise N(0, sigma^2), float32."""
    return (np.random.default_rng(seed).standard_normal(n) * sigma).astype(np.float32)


def pink(seed: int, n: int, rms: float = 0.1) -> np.ndarray:
    """Pink (1/f power) noise: white Gaussian, each rfft bin k scaled by
    k**-0.5 with DC removed, back-transformed, scaled to the given RMS."""
    x = np.random.default_rng(seed).standard_normal(n)
    X = np.fft.rfft(x)
    k = np.arange(X.size, dtype=np.float64)
    k[0] = 1.0
    X *= k ** -0.5
    X[0] = 0.0
    y = np.fft.irfft(X, n)
    y *= rms / max(np.sqrt(np.mean(y * y)), 1e-30)
    return y.astype(np.float32)


# ---------------------------------------------------------------------------
# Job lists and initial factors
# ---------------------------------------------------------------------------
def jobs_fixed(n_src: int, n_dirs_total: int, dirs_per_src: int, seed0: int = 200) -> np.ndarray:
    """Each source at ``dirs_per_src`` distinct directions (drawn without
    replacement with seed seed0 + i); both ears.  Returns int32[n_jobs][2]
    rows (src, filter), filter = 2 * direction + ear."""
    rows = []
    for i in range(n_src):
        ds = np.random.default_rng(seed0 + i).choice(n_dirs_total, size=dirs_per_src, replace=False)
        for d in ds:
            rows.append((i, 2 * int(d)))
            rows.append((i, 2 * int(d) + 1))
    return np.asarray(rows, dtype=np.int32)


def uneven_lengths(seed: int, n_src: int, lo: int = 4096, hi: int = 1 << 20) -> np.ndarray:
    """Source lengths floor(exp(U(ln lo, ln hi)))."""
    u = np.random.default_rng(seed).uniform(math.log(lo), math.log(hi), size=n_src)
    return np.floor(np.exp(u)).astype(np.int64)


def jobs_uneven(seed: int, n_src: int, n_dirs_total: int, max_dirs: int = 8) -> np.ndarray:
    """1..max_dirs distinct directions per source, both ears."""
    rng = np.random.default_rng(seed)
    rows = []
    for i in range(n_src):
        nd = int(rng.integers(1, max_dirs + 1))
        for d in rng.choice(n_dirs_total, size=nd, replace=False):
            rows.append((i, 2 * int(d)))
            rows.append((i, 2 * int(d) + 1))
    return np.asarray(rows, dtype=np.int32)


def random_taps(seed: int, n_filters: int, k: int, lg: int, nnz_min: int | None = None):
    """Random sparse tap tables for parity tests: p int32[F][k] ascending over
    distinct positions in [0, lg), g float32[F][k] >= 0; optionally some rows
    padded with (p=0, g=0) after their real taps."""
    rng = np.random.default_rng(seed)
    p = np.zeros((n_filters, k), dtype=np.int32)
    g = np.zeros((n_filters, k), dtype=np.float32)
    for f in range(n_filters):
        nnz = k if nnz_min is None else int(rng.integers(nnz_min, k + 1))
        nnz = min(nnz, lg)
        pos = np.sort(rng.choice(lg, size=nnz, replace=False))
        p[f, :nnz] = pos
        g[f, :nnz] = rng.uniform(0.0, 1.0, size=nnz).astype(np.float32)
    return p, g


def g0(seed: int, n: int, lg: int) -> np.ndarray:
    """Initial reflection matrix G0 ~ U(0, 1] (Alg. 1's random start)."""
    return 1.0 - np.random.default_rng(seed).uniform(0.0, 1.0, size=(n, lg))


def mlp_params(seed: int, sizes):
    """Initial surrogate parameters: He-uniform weights
    U(-sqrt(6 / k_in), +sqrt(6 / k_in)) and zero biases, float64, as a list
    of (W [k_in][k_out], b [k_out]); the same arrays seed both the library
    and the oracle."""
    rng = np.random.default_rng(seed)
    out = []
    for k_in, k_out in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / k_in)
        out.append((rng.uniform(-lim, lim, (k_in, k_out)), np.zeros(k_out)))
    return out
