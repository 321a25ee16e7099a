"""Plain FP64 CPU oracle for GLS map-making (arXiv:2501.16122, Sec. II).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this module: only the tests, the smoke check and the benchmark's CPU-baseline
leg do.  It shares no code, table or helper with the HIP library; it is slow
and written so that each step can be read against the paper:

* eq. (2)/(8): a sample sees one pixel through the row [1, cos 2psi, sin 2psi]
  (the paper's text once says cos/sin of theta; its equations use 2 theta,
  which is the reading taken here);
* Sec. III-B sizes the reduced pixel-domain array at two or three values per
  sky pixel: besides the I, Q, U map, a polarisation-only map (Q, U; the row
  keeps the two angle columns) and, with one value per pixel, an
  intensity-only map (I; the row is the 1 alone) use the same operators with
  fewer columns;
* eq. (3): d = P s + n;
* eq. (5)/(6): the GLS map solves A x = b with A = P^T N^-1 P, b = P^T N^-1 d;
* eq. (7): the block-Jacobi preconditioner M = (P^T diag(N)^-1 P)^-1, whose
  3x3 blocks are inverted one pixel at a time;
* Sec. II: PCG is the iterative solver (textbook preconditioned conjugate
  gradient, Saad, "Iterative Methods for Sparse Linear Systems", Alg. 9.1).

Readings the paper leaves open (all listed in the design notes): pixels seen
fewer than ``min_hits`` times or whose block has 2-norm condition number above
``cond_max`` are masked and dropped from the unknowns (their samples get a
zero row in P); kept pixels are numbered in ascending pixel order; the
correlated N^-1 is a finite band-Toeplitz section per stationary chunk with
caller-given lags 0..lam-1 and no coupling across chunks; the PCG stops at the
first iterate whose recursively updated residual satisfies
||r_k|| / ||b|| <= tol, starting from x0 = 0.

Every function pins to something other than itself in tests/test_oracle_*.py
(closed forms, brute force on tiny inputs, library reductions, invariants).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.signal


# ---------------------------------------------------------------------------
# Pointing: eq. (2), (8) and the block-diagonal matrix of eq. (7)
# ---------------------------------------------------------------------------

def pointing_weights(psi: np.ndarray):
    """Columns 2 and 3 of a row of P: (cos 2 psi_t, sin 2 psi_t), eq. (2)/(8).

    psi is upcast exactly to FP64 first (FP32-stored angles are the problem
    as stored).
    """
    two_psi = 2.0 * np.asarray(psi, dtype=np.float64)
    return np.cos(two_psi), np.sin(two_psi)


NCOMP = {"IQU": 3, "QU": 2, "I": 1}


def pointing_rows(stokes: str, c: np.ndarray, s: np.ndarray):
    """The columns of P a sample sees for each map form, as per-sample
    arrays: IQU (1, cos 2psi, sin 2psi) as in eq. (8); QU the two angle
    columns alone; I the constant column alone."""
    if stokes == "IQU":
        return (np.ones_like(c), c, s)
    if stokes == "QU":
        return (c, s)
    if stokes == "I":
        return (np.ones_like(c),)
    raise ValueError(f"unknown map form {stokes!r}")


def sample_weights(det_offsets: np.ndarray, det_weight: np.ndarray) -> np.ndarray:
    """Per-sample diagonal of N^-1 for white noise: 1/sigma_d^2 of its detector."""
    det_offsets = np.asarray(det_offsets, dtype=np.int64)
    counts = np.diff(det_offsets)
    return np.repeat(np.asarray(det_weight, dtype=np.float64), counts)


@dataclasses.dataclass
class Pointing:
    """Precomputed pointing elements and preconditioner (Sec. III-A)."""

    pix: np.ndarray          # int32[N_t]
    cos2: np.ndarray         # f64[N_t]
    sin2: np.ndarray         # f64[N_t]
    weight: np.ndarray       # f64[N_t], diag(N)^-1 per sample
    n_pix: int
    hits: np.ndarray         # int64[n_pix]
    blocks: np.ndarray       # f64[n_pix, nc, nc]: P^T diag(N)^-1 P restricted to pixel p
    cond: np.ndarray         # f64[n_pix]: 2-norm condition number (inf if singular)
    mask: np.ndarray         # bool[n_pix]: True = removed from the unknowns
    kept: np.ndarray         # int64[n_kept], ascending pixel indices
    compact: np.ndarray      # int64[n_pix]: position in ``kept`` or -1
    minv: np.ndarray         # f64[n_kept, nc, nc]: inverse blocks (eq. (7))
    sample_k: np.ndarray     # int64[N_t]: compact index of each sample (-1 = masked)
    stokes: str = "IQU"      # map form: "IQU", "QU" or "I" (nc = 3, 2, 1 values per pixel)

    @property
    def ncomp(self) -> int:
        return NCOMP[self.stokes]

    def rows(self):
        return pointing_rows(self.stokes, self.cos2, self.sin2)

    @property
    def n_kept(self) -> int:
        return int(self.kept.size)

    @property
    def n_samples(self) -> int:
        return int(self.pix.size)


def build_pointing(pix, psi, det_offsets, det_weight, n_pix, min_hits=None, cond_max=1e3,
                   stokes="IQU") -> Pointing:
    """Hits, the nc x nc blocks of P^T diag(N)^-1 P, their conditioning, the
    mask and the inverse blocks of the preconditioner (eq. (7)).  min_hits
    defaults to nc, the fewest samples that can make a block invertible.
    psi may be None for the intensity-only form, whose rows do not use it."""
    nc = NCOMP[stokes]
    if min_hits is None:
        min_hits = nc
    pix = np.asarray(pix)
    if psi is None:
        if stokes != "I":
            raise ValueError("the angle is needed unless the map is intensity-only")
        psi = np.zeros(pix.size)
    if pix.size and (pix.min() < 0 or pix.max() >= n_pix):
        raise ValueError("pixel index out of range")
    c, s = pointing_weights(psi)
    w = sample_weights(det_offsets, det_weight)
    if w.size != pix.size:
        raise ValueError("detector offsets do not cover the timeline")
    hits = np.bincount(pix, minlength=n_pix).astype(np.int64)
    # The block of pixel p is sum over its samples of w a a^T, a the row of P.
    a = pointing_rows(stokes, c, s)
    blocks = np.zeros((n_pix, nc, nc))
    for i in range(nc):
        for j in range(nc):
            blocks[:, i, j] = np.bincount(pix, weights=w * a[i] * a[j], minlength=n_pix)
    cond = np.full(n_pix, np.inf)
    seen = hits > 0
    ev = np.linalg.eigvalsh(blocks[seen])
    lo, hi = ev[:, 0], ev[:, -1]
    with np.errstate(divide="ignore", invalid="ignore"):
        cond_seen = np.where(lo > 0, hi / lo, np.inf)
    cond[seen] = cond_seen
    mask = (hits < min_hits) | (cond > cond_max)
    kept = np.flatnonzero(~mask)
    compact = np.full(n_pix, -1, dtype=np.int64)
    compact[kept] = np.arange(kept.size)
    minv = np.linalg.inv(blocks[kept]) if kept.size else np.zeros((0, nc, nc))
    return Pointing(pix=pix, cos2=c, sin2=s, weight=w, n_pix=n_pix, hits=hits,
                    blocks=blocks, cond=cond, mask=mask, kept=kept, compact=compact,
                    minv=minv, sample_k=compact[pix], stokes=stokes)


def mask_margin(pt: Pointing, cond_max=1e3, min_hits=None) -> float:
    """Smallest distance, in decades, between a pixel's condition number and
    the masking threshold (over pixels with enough hits and finite cond).
    A tiny margin means the keep/mask decision hangs on rounding."""
    sel = (pt.hits >= (pt.ncomp if min_hits is None else min_hits)) & np.isfinite(pt.cond)
    if not np.any(sel):
        return np.inf
    return float(np.min(np.abs(np.log10(pt.cond[sel] / cond_max))))


# ---------------------------------------------------------------------------
# Operators: P (eq. (3)/(8)), P^T, N^-1, A = P^T N^-1 P, M (eq. (7))
# ---------------------------------------------------------------------------

def apply_P(pt: Pointing, x: np.ndarray) -> np.ndarray:
    """y_t = I_k + Q_k cos 2psi_t + U_k sin 2psi_t with k the compact index
    of the sample's pixel (the columns the map form keeps); 0 for samples of
    masked pixels."""
    x = np.asarray(x, dtype=np.float64).reshape(-1, pt.ncomp)
    k = pt.sample_k
    ok = k >= 0
    kk = np.where(ok, k, 0)
    y = np.zeros(k.size)
    for j, a in enumerate(pt.rows()):
        y = y + x[kk, j] * a
    return np.where(ok, y, 0.0)


def apply_PT(pt: Pointing, y: np.ndarray) -> np.ndarray:
    """(P^T y)_k = sum over kept samples of pixel k of y_t times the row
    (1, cos, sin), or the columns the map form keeps."""
    y = np.asarray(y, dtype=np.float64)
    ok = pt.sample_k >= 0
    k = pt.sample_k[ok]
    yo = y[ok]
    q = np.zeros((pt.n_kept, pt.ncomp))
    for j, a in enumerate(pt.rows()):
        q[:, j] = np.bincount(k, weights=yo * a[ok], minlength=pt.n_kept)
    return q.reshape(-1)


def apply_ninv_white(pt: Pointing, y: np.ndarray) -> np.ndarray:
    """Diagonal N^-1: scale each sample by its detector's 1/sigma^2."""
    return pt.weight * np.asarray(y, dtype=np.float64)


@dataclasses.dataclass
class ToeplitzNoise:
    """Band-Toeplitz N^-1 applied independently on each stationary chunk."""

    coeff: np.ndarray          # f64[n_filt, lam]: lags 0..lam-1
    chunk_offsets: np.ndarray  # int64[n_chunks + 1]
    chunk_filter: np.ndarray   # int[n_chunks]: which row of coeff each chunk uses

    @property
    def lam(self) -> int:
        return int(self.coeff.shape[1])


def toeplitz_noise(coeff, chunk_offsets, chunk_filter=None) -> ToeplitzNoise:
    coeff = np.atleast_2d(np.asarray(coeff, dtype=np.float64))
    chunk_offsets = np.asarray(chunk_offsets, dtype=np.int64)
    n_chunks = chunk_offsets.size - 1
    if chunk_filter is None:
        chunk_filter = np.zeros(n_chunks, dtype=np.int64)
    return ToeplitzNoise(coeff, chunk_offsets, np.asarray(chunk_filter, dtype=np.int64))


def apply_ninv_toeplitz(noise: ToeplitzNoise, y: np.ndarray) -> np.ndarray:
    """z_i = sum_{j in chunk(i), |i-j| < lam} c_{|i-j|} y_j, chunk by chunk.

    The symmetric kernel [c_{lam-1} .. c_1, c_0, c_1 .. c_{lam-1}] convolved
    with the chunk and cut to the chunk's own support ('same') is exactly the
    finite band section: no wrap-around, no coupling across chunks.
    """
    y = np.asarray(y, dtype=np.float64)
    z = np.zeros_like(y)
    offs = noise.chunk_offsets
    for ci in range(offs.size - 1):
        a, b = int(offs[ci]), int(offs[ci + 1])
        if b <= a:
            continue
        c = noise.coeff[noise.chunk_filter[ci]]
        kern = np.concatenate([c[:0:-1], c])
        if b - a == 1:
            z[a:b] = c[0] * y[a:b]
            continue
        z[a:b] = scipy.signal.oaconvolve(y[a:b], kern, mode="same")
    return z


@dataclasses.dataclass
class CirculantNoise(ToeplitzNoise):
    """Circulant N^-1 on each stationary chunk (Sec. IV): the chunk is taken
    as periodic, and its first row holds the band filter c_0 .. c_{lam-1} and
    its mirror image, so the product is a circular convolution, diagonal in
    the Fourier basis of the chunk.  Chunks must be longer than 2 (lam - 1)."""


def circulant_noise(coeff, chunk_offsets, chunk_filter=None) -> CirculantNoise:
    t = toeplitz_noise(coeff, chunk_offsets, chunk_filter)
    lens = np.diff(t.chunk_offsets)
    if np.any((lens > 0) & (lens <= 2 * (t.lam - 1))):
        raise ValueError("a circulant chunk must be longer than 2 (lam - 1)")
    return CirculantNoise(t.coeff, t.chunk_offsets, t.chunk_filter)


def apply_ninv_circulant(noise: CirculantNoise, y: np.ndarray) -> np.ndarray:
    """z = h (*) y per chunk, the circular convolution with the chunk's first
    row h (h_tau = h_{n - tau} = c_tau for tau < lam, 0 elsewhere), by the
    FFT of the chunk."""
    y = np.asarray(y, dtype=np.float64)
    z = np.zeros_like(y)
    offs = noise.chunk_offsets
    for ci in range(offs.size - 1):
        a, b = int(offs[ci]), int(offs[ci + 1])
        n = b - a
        if n <= 0:
            continue
        c = noise.coeff[noise.chunk_filter[ci]]
        h = np.zeros(n)
        h[:c.size] = c
        if c.size > 1:
            h[n - c.size + 1:] = c[:0:-1]
        z[a:b] = np.fft.irfft(np.fft.rfft(y[a:b]) * np.fft.rfft(h), n)
    return z


@dataclasses.dataclass
class TemplateNoise:
    """A general weight W of eq. (4) built from filtering templates (Sec.
    IV): the white weights w (1/sigma_d^2 per detector) with polynomial
    baselines marginalised on each interval,
        W = N_w^-1 - N_w^-1 T (T^T N_w^-1 T)^-1 T^T N_w^-1,
    where T holds, for every interval, the polynomials of degree < order in
    the sample position (columns zero outside the interval).  Intervals do
    not cross detector starts, so w is constant on each and W acts there as
    w (I - T (T^T T)^-1 T^T); samples outside every interval get w alone."""

    interval_offsets: np.ndarray  # int64[n_intervals + 1]
    orders: np.ndarray            # int[n_intervals]: degrees 0 .. order-1 per interval (0 = none)


def template_noise(interval_offsets, order) -> TemplateNoise:
    """order: one value for every interval, or one per interval."""
    offs = np.asarray(interval_offsets, dtype=np.int64)
    orders = np.broadcast_to(np.asarray(order, dtype=np.int64), (max(offs.size - 1, 0),)).copy()
    if np.any(np.diff(offs) < 0) or np.any(orders < 0):
        raise ValueError("bad template intervals or order")
    return TemplateNoise(offs, orders)


def template_matrix(n: int, order: int) -> np.ndarray:
    """T of one interval of n samples: Legendre polynomials of degree
    < min(order, n) at n equispaced positions spanning [-1, 1] (any basis of
    the same polynomials gives the same W)."""
    k = min(order, n)
    u = np.linspace(-1.0, 1.0, n) if n > 1 else np.zeros(1)
    return np.polynomial.legendre.legvander(u, k - 1) if k > 0 else np.zeros((n, 0))


def apply_w_templates(pt: Pointing, noise: TemplateNoise, y: np.ndarray) -> np.ndarray:
    """z = W y with W of TemplateNoise: per interval w (y - T (T^T T)^-1 T^T y)."""
    y = np.asarray(y, dtype=np.float64)
    z = pt.weight * y
    offs = noise.interval_offsets
    for ii in range(offs.size - 1):
        a, b = int(offs[ii]), int(offs[ii + 1])
        order = int(noise.orders[ii])
        if b <= a or order == 0:
            continue
        if np.any(pt.weight[a:b] != pt.weight[a]):
            raise ValueError("a template interval must lie within one detector")
        T = template_matrix(b - a, order)
        ya = y[a:b]
        coef = np.linalg.solve(T.T @ T, T.T @ ya)
        z[a:b] = pt.weight[a:b] * (ya - T @ coef)
    return z


def apply_ninv(pt: Pointing, noise, y):
    if noise is None:
        return apply_ninv_white(pt, y)
    if isinstance(noise, TemplateNoise):
        return apply_w_templates(pt, noise, y)
    if isinstance(noise, CirculantNoise):
        return apply_ninv_circulant(noise, y)
    return apply_ninv_toeplitz(noise, y)


def apply_A(pt: Pointing, noise, x):
    """A x = P^T N^-1 P x (eq. (6))."""
    return apply_PT(pt, apply_ninv(pt, noise, apply_P(pt, x)))


def rhs(pt: Pointing, noise, d):
    """b = P^T N^-1 d (eq. (6))."""
    return apply_PT(pt, apply_ninv(pt, noise, d))


def apply_M(pt: Pointing, r: np.ndarray) -> np.ndarray:
    """z = M r with M the block-diagonal inverse of eq. (7)."""
    r = np.asarray(r, dtype=np.float64).reshape(-1, pt.ncomp)
    return np.einsum("kij,kj->ki", pt.minv, r).reshape(-1)


# ---------------------------------------------------------------------------
# PCG (Sec. II) and the solve of eq. (5)/(6)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class PCGInfo:
    iters: int
    converged: bool
    breakdown: bool
    rel_resid: float              # recursively updated residual at exit
    true_rel_resid: float         # ||b - A x|| / ||b|| recomputed at exit
    history: list                 # ||r_k|| / ||b|| for k = 0..iters


def pcg(apply_a, apply_m, b, tol=1e-10, max_iter=2000, fixed_iters=None, x0=None):
    """Preconditioned conjugate gradient (Saad, Alg. 9.1).

    Stops at the first k with ||r_k|| / ||b|| <= tol (r_k the recursively
    updated residual), or after exactly ``fixed_iters`` iterations when that
    is given (no early stop).  Breakdown: p^T A p <= 0 or a non-finite value.
    """
    b = np.asarray(b, dtype=np.float64)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:  # A x = 0 with A SPD: x = 0, whatever the start
        return np.zeros_like(b), PCGInfo(0, True, False, 0.0, 0.0, [0.0])
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply_a(x) if x0 is not None else b.copy()
    z = apply_m(r)
    p = z.copy()
    rho = float(r @ z)
    hist = [float(np.linalg.norm(r)) / bnorm]
    limit = max_iter if fixed_iters is None else fixed_iters
    k = 0
    converged = fixed_iters is None and hist[0] <= tol
    breakdown = False
    while k < limit and not converged:
        q = apply_a(p)
        pq = float(p @ q)
        if not np.isfinite(pq) or pq <= 0.0:
            breakdown = True
            break
        alpha = rho / pq
        x = x + alpha * p
        r = r - alpha * q
        k += 1
        rel = float(np.linalg.norm(r)) / bnorm
        hist.append(rel)
        if not np.isfinite(rel):
            breakdown = True
            break
        if fixed_iters is None and rel <= tol:
            converged = True
            break
        z = apply_m(r)
        rho_new = float(r @ z)
        beta = rho_new / rho
        rho = rho_new
        p = z + beta * p
    true_rel = float(np.linalg.norm(b - apply_a(x))) / bnorm
    if fixed_iters is not None:
        converged = hist[-1] <= tol
    return x, PCGInfo(k, converged, breakdown, hist[-1], true_rel, hist)


def expand(pt: Pointing, x: np.ndarray) -> np.ndarray:
    """Compact unknowns -> full-grid f64[n_pix, nc], 0 at masked pixels."""
    out = np.zeros((pt.n_pix, pt.ncomp))
    out[pt.kept] = np.asarray(x, dtype=np.float64).reshape(-1, pt.ncomp)
    return out


def solve(pt: Pointing, noise, d, tol=1e-10, max_iter=2000, fixed_iters=None):
    """GLS map of eq. (5) on the kept pixels by PCG; returns (map, info, x)."""
    b = rhs(pt, noise, d)
    x, info = pcg(lambda v: apply_A(pt, noise, v), lambda v: apply_M(pt, v), b,
                  tol=tol, max_iter=max_iter, fixed_iters=fixed_iters)
    return expand(pt, x), info, x


def binned_map(pt: Pointing, d) -> np.ndarray:
    """White-noise GLS map: per kept pixel, B_p^-1 (sum w a d).  With diagonal
    N^-1 the matrix A is block-diagonal (eq. (7)), so this is the exact
    solution of eq. (5)."""
    b = rhs(pt, None, d).reshape(-1, pt.ncomp)
    x = np.linalg.solve(pt.blocks[pt.kept], b[..., None])[..., 0]
    return x.reshape(-1)


def rel_l2_per_stokes(m, m_ref, kept=None, ncomp=3):
    """||m - m_ref|| / ||m_ref|| separately for each Stokes parameter of the
    map (I, Q, U; or those of the map form's ncomp) over kept pixels."""
    m = np.asarray(m, dtype=np.float64).reshape(-1, ncomp)
    m_ref = np.asarray(m_ref, dtype=np.float64).reshape(-1, ncomp)
    if kept is not None:
        m, m_ref = m[kept], m_ref[kept]
    num = np.linalg.norm(m - m_ref, axis=0)
    den = np.linalg.norm(m_ref, axis=0)
    return num / np.where(den > 0, den, 1.0)
