"""Seeded synthetic inputs for GLS map-making (scan, sky, noise, noise model).

This module draws and shapes random inputs only.  It holds none of the
map-making arithmetic: it never projects a map into a timeline (eq. (2)/(3)),
never bins, never inverts a block and never applies a noise weighting.  The
timeline ``d = P m + n`` is formed by the caller with whichever operator it is
testing or timing; the pieces it needs (pixel indices, angles, the input map,
the noise realisation and the band-Toeplitz coefficients of N^-1) all come
from here, identically for every consumer.

Scan law and noise recipe (the paper fixes none of them; it simulates an
unnamed CMB polarization experiment, abstract and Sec. III-B):

* detector d, sample t = 0..n_samp-1 (integer sample index, detector-major
  layout, so detector d owns samples [d*n_samp, (d+1)*n_samp));
* x(t) = (W/2) (1 + sin(2 pi t / t_x)),  y(t) = floor(H t / n_samp);
* seeded per-detector offsets dx, dy ~ U[-2, 2] px and angle phi ~ U[0, pi);
* pixel column floor(x + dx), row floor(y + dy), each clamped into the grid,
  pixel = row * W + column (int32, row-major);
* psi(t) = 2 pi t / t_psi + phi  (the angle theta_t of eq. (2));
* sky I ~ N(0, 100^2), Q, U ~ N(0, 1) per pixel;
* noise: white N(0, sigma^2), or 1/f with PSD sigma^2 (1 + (f_knee/f)^alpha)
  made by filtering white noise in the Fourier domain over each detector's
  whole timeline (zero-frequency amplitude set to 0), sample rate fs;
* N^-1 model for correlated noise: per stationary chunk of ``chunk`` samples,
  lags 0..lam-1 of the inverse-PSD autocorrelation on the chunk's frequency
  grid (1/P(0) := 0), optionally Bartlett-tapered (w_tau = 1 - tau/lam).

Seeds: ``SeedSequence([16122, config_id, stream])`` with stream 0 = detector
offsets/angles, 1 = sky, 2 = noise (spawned once per detector), 3 = batch
member sizes, 4 = serving arrivals.
"""
from __future__ import annotations

import dataclasses
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import scipy.fft as sfft

ROOT_SEED = 16122
STREAM_DETECTORS, STREAM_SKY, STREAM_NOISE, STREAM_BATCH, STREAM_SERVE = 0, 1, 2, 3, 4


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic map-making problem (sizes, scan law, noise model)."""

    name: str
    config_id: int
    width: int
    height: int
    n_det: int
    n_samp: int                 # samples per detector
    t_x: float = 600.0          # scan period along x, in samples
    t_psi: float = 200.0        # polarisation-angle period, in samples
    fs: float = 20.0            # sample rate (Hz); only enters the frequency axis
    sigma: float = 1.0          # white-noise level
    noise: str = "white"        # "white" | "oneoverf" | "none"
    fknee: float = 0.1
    alpha: float = 1.5
    chunk: int = 0              # stationary chunk length; 0 = diagonal N^-1
    lam: int = 0                # band half-width (number of lags) of N^-1
    taper: bool = True
    min_hits: int = 3
    cond_max: float = 1e3
    precision: str = "f64"      # storage of psi and d: "f64" | "f32"

    @property
    def n_pix(self) -> int:
        return self.width * self.height

    @property
    def n_samples(self) -> int:
        return self.n_det * self.n_samp

    @property
    def toeplitz(self) -> bool:
        return self.chunk > 0 and self.lam > 0

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


# The configurations of the headline workloads (sizes as stated for them).
C1_BINNED = Workload("binned_64x64_4x2^18_white", 1, 64, 64, 4, 1 << 18, t_psi=200.0)
C2_GLS = Workload("gls_512x512_64x2^22_1overf_toeplitz4096", 2, 512, 512, 64, 1 << 22,
                  t_psi=6000.0, noise="oneoverf", chunk=1 << 20, lam=4096)
# Precision form of C1: the same draws as C1 (same config id), stored in FP32.
C3_PRECISION = C1_BINNED.replace(name="binned_64x64_4x2^18_white_f32", precision="f32")
# One GPU's share of C2 under sample sharding over 8 devices (8 of 64 detectors).
C2_SHARD = C2_GLS.replace(name="gls_512x512_8x2^22_1overf_toeplitz4096", n_det=8)

# Multi-RHS form: 8 seeded noise realisations sharing one pointing (the
# realisation index enters the noise seed), FP32 storage with FP64 refinement.
C4_MULTI = Workload("multirhs_512x512_32x2^22_x8_1overf_toeplitz4096_f32", 4, 512, 512, 32, 1 << 22,
                    t_psi=6000.0, noise="oneoverf", chunk=1 << 20, lam=4096, precision="f32")

CONFIGS = {w.name: w for w in (C1_BINNED, C2_GLS, C3_PRECISION, C2_SHARD, C4_MULTI)}

# The same workloads as JSON files (configs/), with the solve options they
# are run with and a reference to the readings file, which lists every point
# the paper leaves open and the fields that carry its value.
CONFIG_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "configs")
SOLVE_KEYS = ("tol", "max_iter", "check_every", "autotune", "mixed", "bj_start", "inner_tol", "max_outer")


def config_path(name_or_path: str) -> str:
    """A workload file by path, or by name under configs/ (with or without
    the .json suffix)."""
    if os.path.isfile(name_or_path):
        return name_or_path
    p = os.path.join(CONFIG_DIR, name_or_path if name_or_path.endswith(".json") else name_or_path + ".json")
    if not os.path.isfile(p):
        raise FileNotFoundError(f"no workload file {name_or_path!r} (looked in {CONFIG_DIR})")
    return p


def load_config(name_or_path: str):
    """(Workload, solve options) from a workload file: "workload" holds every
    field of Workload and no other, "solve" only names of the solve options."""
    import json
    with open(config_path(name_or_path)) as f:
        d = json.load(f)
    wl = d.get("workload")
    if not isinstance(wl, dict):
        raise ValueError("a workload file needs a 'workload' object")
    names = {f.name for f in dataclasses.fields(Workload)}
    missing, extra = sorted(names - set(wl)), sorted(set(wl) - names)
    if missing or extra:
        raise ValueError(f"workload fields missing {missing}, unknown {extra}")
    solve = dict(d.get("solve", {}))
    bad = sorted(set(solve) - set(SOLVE_KEYS))
    if bad:
        raise ValueError(f"unknown solve options {bad}")
    return Workload(**wl), solve


def config_dict(w: Workload, solve: dict, description: str = "") -> dict:
    """The JSON form of a workload and its solve options (load_config's inverse)."""
    return {"name": w.name, "description": description, "workload": dataclasses.asdict(w), "solve": dict(solve),
            "readings": "readings.json"}


def batch_workloads(n: int = 16, config_id: int = 4, det=(8, 128), samples=(1 << 20, 1 << 23),
                    side=(128, 1024)) -> list:
    """n independent solves of uneven size: detectors, samples per detector
    and grid side each log-uniform over the given ranges (stream 3); 1/f
    noise with the band-Toeplitz N^-1 of the GLS workload, FP32 storage."""
    rng = _rng(config_id, STREAM_BATCH)

    def logu(lo, hi):
        return int(round(float(np.exp(rng.uniform(np.log(lo), np.log(hi))))))

    out = []
    for i in range(n):
        nd, ns, sd = logu(*det), logu(*samples), logu(*side)
        out.append(Workload(f"batch{i}_{sd}x{sd}_{nd}x{ns}", config_id * 1000 + i, sd, sd, nd, ns, t_psi=6000.0,
                            noise="oneoverf", chunk=1 << 20, lam=4096, precision="f32"))
    return out


def _rng(config_id: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([ROOT_SEED, config_id, stream]))


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def detector_params(w: Workload):
    """Per-detector (dx, dy, phi): offsets U[-2, 2] px and angle U[0, pi)."""
    rng = _rng(w.config_id, STREAM_DETECTORS)
    dx = rng.uniform(-2.0, 2.0, w.n_det)
    dy = rng.uniform(-2.0, 2.0, w.n_det)
    phi = rng.uniform(0.0, np.pi, w.n_det)
    return dx, dy, phi


def det_offsets(w: Workload) -> np.ndarray:
    """int64[n_det + 1]: detector d owns samples [off[d], off[d+1])."""
    return np.arange(w.n_det + 1, dtype=np.int64) * w.n_samp


def det_weight(w: Workload) -> np.ndarray:
    """Per-detector white-noise weight 1/sigma_d^2 (sigma_d = sigma for all)."""
    return np.full(w.n_det, 1.0 / (w.sigma * w.sigma))


def _scan_one(w: Workload, d: int, dx, dy, phi, pix_out, psi_out):
    t = np.arange(w.n_samp, dtype=np.float64)
    x = (0.5 * w.width) * (1.0 + np.sin((2.0 * np.pi / w.t_x) * t))
    y = np.floor((w.height * t) / w.n_samp)
    col = np.clip(np.floor(x + dx[d]), 0, w.width - 1).astype(np.int64)
    row = np.clip(np.floor(y + dy[d]), 0, w.height - 1).astype(np.int64)
    pix_out[:] = (row * w.width + col).astype(np.int32)
    psi_out[:] = (2.0 * np.pi / w.t_psi) * t + phi[d]


def pointing(w: Workload):
    """(pix int32[N_t], psi f64[N_t]) for the whole detector-major timeline.

    psi is returned in FP64; ``storage`` rounds it for FP32 forms.
    """
    dx, dy, phi = detector_params(w)
    pix = np.empty(w.n_samples, dtype=np.int32)
    psi = np.empty(w.n_samples, dtype=np.float64)
    n = w.n_samp

    def job(d):
        _scan_one(w, d, dx, dy, phi, pix[d * n:(d + 1) * n], psi[d * n:(d + 1) * n])

    if w.n_det > 1 and w.n_samples >= (1 << 20):
        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(job, range(w.n_det)))
    else:
        for d in range(w.n_det):
            job(d)
    return pix, psi


def sky(w: Workload) -> np.ndarray:
    """f64[n_pix, 3] input map: columns I, Q, U."""
    rng = _rng(w.config_id, STREAM_SKY)
    m = np.empty((w.n_pix, 3))
    m[:, 0] = rng.normal(0.0, 100.0, w.n_pix)
    m[:, 1] = rng.normal(0.0, 1.0, w.n_pix)
    m[:, 2] = rng.normal(0.0, 1.0, w.n_pix)
    return m


def _oneoverf_amplitude(n: int, fs: float, fknee: float, alpha: float) -> np.ndarray:
    f = np.arange(n // 2 + 1, dtype=np.float64) * (fs / n)
    amp = np.zeros_like(f)
    amp[1:] = np.sqrt(1.0 + (fknee / f[1:]) ** alpha)
    return amp


def noise(w: Workload) -> np.ndarray:
    """f64[N_t] noise realisation (zeros for noise == "none")."""
    if w.noise not in ("white", "oneoverf", "none"):
        raise ValueError(f"unknown noise kind {w.noise!r}")
    out = np.zeros(w.n_samples)
    if w.noise == "none":
        return out
    seqs = np.random.SeedSequence([ROOT_SEED, w.config_id, STREAM_NOISE]).spawn(w.n_det)
    n = w.n_samp
    amp = _oneoverf_amplitude(n, w.fs, w.fknee, w.alpha) if w.noise == "oneoverf" else None

    def job(d):
        white = np.random.default_rng(seqs[d]).standard_normal(n)
        if amp is None:
            out[d * n:(d + 1) * n] = w.sigma * white
        else:
            spec = sfft.rfft(white)
            spec *= amp
            out[d * n:(d + 1) * n] = w.sigma * sfft.irfft(spec, n=n)

    if w.n_det > 1 and w.n_samples >= (1 << 20):
        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(job, range(w.n_det)))
    else:
        for d in range(w.n_det):
            job(d)
    return out


def toeplitz_coeff(w: Workload, taper: bool | None = None) -> np.ndarray:
    """f64[lam] lags 0..lam-1 of the band-Toeplitz model of N^-1 for one chunk.

    Inverse-PSD autocorrelation on the chunk's frequency grid, 1/P(0) := 0,
    times the Bartlett window 1 - tau/lam when tapered (the taper keeps every
    finite section positive definite: its symbol is a Fejer-smoothed 1/P).
    """
    if not w.toeplitz:
        raise ValueError("workload has no band-Toeplitz noise model")
    taper = w.taper if taper is None else taper
    n = w.chunk
    f = np.arange(n // 2 + 1, dtype=np.float64) * (w.fs / n)
    inv_p = np.zeros_like(f)
    inv_p[1:] = 1.0 / (w.sigma ** 2 * (1.0 + (w.fknee / f[1:]) ** w.alpha))
    c = sfft.irfft(inv_p, n=n)[: w.lam].copy()
    if taper:
        c *= 1.0 - np.arange(w.lam, dtype=np.float64) / w.lam
    return c


def chunk_offsets(w: Workload) -> np.ndarray:
    """int64[n_chunks + 1] stationary chunks of ``w.chunk`` samples.

    Chunks never cross a detector start; a detector's last chunk may be short.
    """
    offs = [0]
    for d in range(w.n_det):
        start, end = d * w.n_samp, (d + 1) * w.n_samp
        s = start
        while s < end:
            s = min(s + w.chunk, end)
            offs.append(s)
    return np.asarray(offs, dtype=np.int64)


def storage(w: Workload, a: np.ndarray) -> np.ndarray:
    """Round a timeline-domain array to the workload's storage precision.

    FP32 forms round psi and d once (round-to-nearest-even); those rounded
    values are the problem that every consumer then solves.
    """
    if w.precision == "f32":
        return np.ascontiguousarray(a, dtype=np.float32)
    if w.precision == "f64":
        return np.ascontiguousarray(a, dtype=np.float64)
    raise ValueError(f"unknown precision {w.precision!r}")
