"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bar: integer products of the build (hits, mask, compact, kept) bit-exact;
FP64 operators and maps within the tolerances written next to each check
(derived from the arithmetic: FP64 FFT round-off of the Toeplitz section is
O(log L * eps) relative to the norm of its output, and map parity is checked
per Stokes component at a fixed iteration count).
"""
import numpy as np
import pytest

import oracle.mapmaking as oracle
from paper_2501_16122_amd import synth
from parity_util import err as rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _b():
    from paper_2501_16122_amd import binding
    return binding


DEV = "cuda:0"

# several pointing tiles and FFT tiles with ragged tails: 3 detectors of
# 3*2^16 + 777 samples, chunks of 2^15 + 123 samples, a 128^2 grid
RAGGED = synth.Workload("ragged_128x128_3x197385", 931, 128, 128, 3, 3 * (1 << 16) + 777, t_psi=1500.0,
                        noise="oneoverf", chunk=(1 << 15) + 123, lam=512)


class Problem:
    def __init__(self, w: synth.Workload, with_d=True):
        self.w = w
        pix, psi = synth.pointing(w)
        self.pix = pix
        self.psi = synth.storage(w, psi)
        self.offs = synth.det_offsets(w)
        self.wdet = synth.det_weight(w)
        self.opt = oracle.build_pointing(self.pix, self.psi, self.offs, self.wdet, w.n_pix, w.min_hits, w.cond_max)
        self.noise = None
        if w.toeplitz:
            self.coeff = synth.toeplitz_coeff(w)
            self.chunks = synth.chunk_offsets(w)
            self.noise = oracle.toeplitz_noise(self.coeff, self.chunks)
        if with_d:
            m = synth.sky(w)[self.opt.kept].reshape(-1)
            self.d = synth.storage(w, oracle.apply_P(self.opt, m) + synth.noise(w))

    def device(self):
        b = _b()
        self.t_pix = torch.from_numpy(self.pix).to(DEV)
        self.t_psi = torch.from_numpy(self.psi).to(DEV)
        self.pt = b.Pointing(self.t_pix, self.t_psi, self.offs, self.wdet, self.w.n_pix, self.w.min_hits,
                             self.w.cond_max)
        if self.w.toeplitz:
            self.nz = b.Noise.toeplitz(self.coeff, self.chunks, DEV)
        else:
            self.nz = b.Noise.white(self.wdet, DEV)
        if hasattr(self, "d"):
            self.t_d = torch.from_numpy(self.d).to(DEV)
        return self


@pytest.fixture(scope="module")
def ragged():
    return Problem(RAGGED).device()


@pytest.fixture(scope="module")
def binned():
    return Problem(synth.C1_BINNED).device()


def _check_build(P):
    out = P.pt.export()
    torch.cuda.synchronize()
    o = P.opt
    assert P.pt.n_kept == o.n_kept
    assert np.array_equal(out["hits"].cpu().numpy(), o.hits.astype(np.int32))
    assert np.array_equal(out["mask"].cpu().numpy().astype(bool), o.mask)
    assert np.array_equal(out["compact"].cpu().numpy(), o.compact.astype(np.int32))
    assert np.array_equal(out["kept"].cpu().numpy(), o.kept.astype(np.int32))
    minv = out["minv"].cpu().numpy()
    assert rel_err(minv, o.minv, 9) < 1e-12


def test_build_bit_exact_ragged(ragged):
    _check_build(ragged)
    assert oracle.mask_margin(ragged.opt) > 1e-9


def test_build_bit_exact_binned(binned):
    _check_build(binned)
    assert oracle.mask_margin(binned.opt) > 1e-9


def test_build_masks_and_edge_pixels():
    # few hits, singular blocks (constant angle) and unseen pixels on a tiny grid
    b = _b()
    rng = np.random.default_rng(5)
    n = 3000
    pix = rng.integers(0, 40, n).astype(np.int32)
    pix[pix == 7] = 8
    pix[:2] = 7                                  # seen twice
    psi = rng.uniform(0, 7, n)
    psi[pix == 9] = 0.25                         # one angle only: singular block
    offs = np.array([0, 1000, 1000, 3000])       # includes an empty detector
    w = np.array([1.0, 2.0, 0.5])
    o = oracle.build_pointing(pix, psi, offs, w, 41)
    pt = b.Pointing(torch.from_numpy(pix).to(DEV), torch.from_numpy(psi).to(DEV), offs, w, 41)
    ex = pt.export()
    assert np.array_equal(ex["hits"].cpu().numpy(), o.hits)
    assert np.array_equal(ex["mask"].cpu().numpy().astype(bool), o.mask)
    assert o.mask[7] and o.mask[9] and o.mask[40]
    assert np.array_equal(ex["compact"].cpu().numpy(), o.compact)


def test_build_rejects_bad_pixel():
    b = _b()
    pix = torch.tensor([0, 1, 5], dtype=torch.int32, device=DEV)
    psi = torch.zeros(3, dtype=torch.float64, device=DEV)
    with pytest.raises(b.MapMakerError) as ei:
        b.Pointing(pix, psi, [0, 3], [1.0], 5)
    assert ei.value.code == b.MM_EINVAL


def test_build_rejects_bad_angle():
    b = _b()
    pix = torch.tensor([0, 1, 1], dtype=torch.int32, device=DEV)
    for bad in (float("nan"), float("inf"), 3e8):
        psi = torch.tensor([0.1, bad, 0.2], dtype=torch.float64, device=DEV)
        with pytest.raises(b.MapMakerError) as ei:
            b.Pointing(pix, psi, [0, 3], [1.0], 5)
        assert ei.value.code == b.MM_EINVAL


def test_P_PT_white_ninv(ragged):
    b = _b()
    P = ragged
    rng = np.random.default_rng(11)
    x = rng.normal(size=3 * P.opt.n_kept)
    y = rng.normal(size=P.w.n_samples)
    tx, ty = torch.from_numpy(x).to(DEV), torch.from_numpy(y).to(DEV)
    yp = b.apply_P(P.pt, tx).cpu().numpy()
    assert rel_err(yp, oracle.apply_P(P.opt, x)) < 1e-14
    q = b.apply_PT(P.pt, ty).cpu().numpy()
    assert rel_err(q, oracle.apply_PT(P.opt, y), 3) < 1e-13
    nzw = b.Noise.white(P.wdet * np.array([1.0, 0.5, 2.0]), DEV)
    z = b.apply_Ninv(nzw, P.pt, ty).cpu().numpy()
    wt = np.repeat(P.wdet * np.array([1.0, 0.5, 2.0]), np.diff(P.offs))
    assert np.array_equal(z, wt * y)
    # adjoint identity on the device operators
    lhs = float(np.dot(yp, y))
    rhs_ = float(np.dot(x, q))
    assert abs(lhs - rhs_) <= 1e-12 * (abs(lhs) + 1)


def test_fused_white_matches_oracle(binned):
    b = _b()
    P = binned
    x = np.random.default_rng(12).normal(size=3 * P.opt.n_kept)
    q = b.apply_A(P.pt, P.nz, torch.from_numpy(x).to(DEV)).cpu().numpy()
    assert rel_err(q, oracle.apply_A(P.opt, None, x), 3) < 1e-13


@pytest.mark.parametrize("lam", [1, 7, 64, 512, 4096])
def test_toeplitz_ninv_matches_oracle(lam):
    b = _b()
    w = RAGGED.replace(lam=lam, n_det=2, n_samp=(1 << 16) + 333, chunk=(1 << 14) + 57)
    P = Problem(w, with_d=False)
    y = np.random.default_rng(lam).normal(size=w.n_samples) * 10
    P.device()
    z = b.apply_Ninv(P.nz, P.pt, torch.from_numpy(y).to(DEV)).cpu().numpy()
    zr = oracle.apply_ninv_toeplitz(P.noise, y)
    assert rel_err(z, zr) < 1e-13
    assert np.max(np.abs(z - zr)) < 1e-12 * np.max(np.abs(zr))


def test_toeplitz_uneven_chunks_and_filters():
    # chunks shorter than a tile, a 1-sample chunk, a gap no chunk covers,
    # and two filters
    b = _b()
    n = 60000
    rng = np.random.default_rng(21)
    pix = rng.integers(0, 50, n).astype(np.int32)
    psi = rng.uniform(0, 6, n)
    offs_det = np.array([0, 30000, n])
    chunks = np.array([0, 1, 5000, 30000, 30017, 50000])  # samples 50000.. uncovered
    filt = np.array([0, 1, 0, 1, 1], dtype=np.int32)
    coeff = rng.normal(size=(2, 300)) * np.array([[1.0], [0.3]])
    y = rng.normal(size=n)
    pt = b.Pointing(torch.from_numpy(pix).to(DEV), torch.from_numpy(psi).to(DEV), offs_det, [1.0, 1.0], 50)
    nz = b.Noise.toeplitz(coeff, chunks, DEV, chunk_filter=filt)
    z = b.apply_Ninv(nz, pt, torch.from_numpy(y).to(DEV)).cpu().numpy()
    zr = oracle.apply_ninv_toeplitz(oracle.toeplitz_noise(coeff, chunks, filt), y)
    assert rel_err(z, zr) < 1e-13
    assert np.all(z[50000:] == 0)


def test_toeplitz_chunk_crossing_detector_rejected():
    b = _b()
    pix = torch.zeros(100, dtype=torch.int32, device=DEV)
    psi = torch.linspace(0, 3, 100, dtype=torch.float64, device=DEV)
    pt = b.Pointing(pix, psi, [0, 50, 100], [1.0, 1.0], 1)
    nz = b.Noise.toeplitz(np.ones(4), [0, 60, 100], DEV)
    with pytest.raises(b.MapMakerError):
        b.apply_Ninv(nz, pt, torch.zeros(100, dtype=torch.float64, device=DEV))


def test_fused_toeplitz_and_rhs_match_oracle(ragged):
    b = _b()
    P = ragged
    x = np.random.default_rng(13).normal(size=3 * P.opt.n_kept)
    q = b.apply_A(P.pt, P.nz, torch.from_numpy(x).to(DEV)).cpu().numpy()
    assert rel_err(q, oracle.apply_A(P.opt, P.noise, x), 3) < 1e-12
    bb = b.rhs(P.pt, P.nz, P.t_d).cpu().numpy()
    assert rel_err(bb, oracle.rhs(P.opt, P.noise, P.d), 3) < 1e-12
    # the fused pass equals the composition of the standalone operators
    y = b.apply_P(P.pt, torch.from_numpy(x).to(DEV))
    z = b.apply_Ninv(P.nz, P.pt, y)
    q2 = b.apply_PT(P.pt, z).cpu().numpy()
    assert rel_err(q, q2, 3) < 1e-13


def test_apply_M_and_expand(ragged):
    b = _b()
    P = ragged
    r = np.random.default_rng(14).normal(size=3 * P.opt.n_kept)
    z = b.apply_M(P.pt, torch.from_numpy(r).to(DEV)).cpu().numpy()
    assert rel_err(z, oracle.apply_M(P.opt, r), 3) < 1e-13
    full = b.expand_map(P.pt, torch.from_numpy(r).to(DEV)).cpu().numpy().reshape(-1, 3)
    assert np.array_equal(full, oracle.expand(P.opt, r))


def test_white_solve_binned_config(binned):
    b = _b()
    P = binned
    s = b.Solver(P.pt, P.nz, tol=1e-10)
    out = s.solve(P.t_d, history=True)
    m_ref, info, x_ref = oracle.solve(P.opt, None, P.d, tol=1e-10)
    assert out["info"]["converged"] == 1 and out["info"]["iters"] == info.iters == 1
    x = out["x"].cpu().numpy()
    assert np.all(oracle.rel_l2_per_stokes(x, x_ref) < 1e-10)
    assert np.all(oracle.rel_l2_per_stokes(x, oracle.binned_map(P.opt, P.d)) < 1e-10)
    full = out["map"].cpu().numpy().reshape(-1, 3)
    assert np.all(full[P.opt.mask] == 0)


def test_toeplitz_solve_fixed_iterations(ragged):
    b = _b()
    P = ragged
    _, info_tol, _ = oracle.solve(P.opt, P.noise, P.d, tol=1e-10)
    k = info_tol.iters
    assert 5 < k < 400
    _, info_k, x_ref = oracle.solve(P.opt, P.noise, P.d, fixed_iters=k)
    s = b.Solver(P.pt, P.nz, fixed_iter=k)
    out = s.solve(P.t_d, history=True)
    assert out["info"]["iters"] == k
    x = out["x"].cpu().numpy()
    err = oracle.rel_l2_per_stokes(x, x_ref)
    assert np.all(err < 1e-10), err
    # residual histories agree too
    h = out["history"]
    assert np.allclose(h[: k + 1], info_k.history[: k + 1], rtol=1e-6, atol=1e-14)
    # and the tolerance-driven solve stops at the same iteration
    s2 = b.Solver(P.pt, P.nz, tol=1e-10)
    out2 = s2.solve(P.t_d)
    assert out2["info"]["converged"] == 1
    assert abs(out2["info"]["iters"] - k) <= 1
    assert out2["info"]["true_rel_resid"] < 1e-9


def test_fused_toeplitz_with_stored_weights(ragged):
    # the precomputed (cos, sin) path gives the same operator
    b = _b()
    P = ragged
    x = np.random.default_rng(15).normal(size=3 * P.opt.n_kept)
    tx = torch.from_numpy(x).to(DEV)
    q0 = b.apply_A(P.pt, P.nz, tx).cpu().numpy()
    P.pt.attach_weights()
    try:
        # the stored weight is u = tan psi; the row's (cos 2psi, sin 2psi)
        # is ((1 - u^2), 2u) / (1 + u^2)
        u = P.pt.weights.cpu().numpy()
        assert u.shape == (P.w.n_samples,)
        assert np.max(np.abs((1 - u * u) / (1 + u * u) - P.opt.cos2)) < 2e-15
        assert np.max(np.abs(2 * u / (1 + u * u) - P.opt.sin2)) < 2e-15
        q1 = b.apply_A(P.pt, P.nz, tx).cpu().numpy()
        bb = b.rhs(P.pt, P.nz, P.t_d).cpu().numpy()
    finally:
        P.pt.detach_weights()
    assert rel_err(q1, oracle.apply_A(P.opt, P.noise, x), 3) < 1e-12
    assert rel_err(q1, q0, 3) < 1e-13
    assert rel_err(bb, oracle.rhs(P.opt, P.noise, P.d), 3) < 1e-12


def _mixed_problem(w):
    # FP32 storage of psi and d: the oracle solves the exact FP64 upcast of the
    # same rounded arrays (the rounded values are the problem)
    return Problem(w.replace(precision="f32")).device()


def test_precision_form_binned_refined():
    # precision form of the binned configuration: FP32 psi/d/timeline
    # arithmetic, FP64 refinement to 1e-10; white noise, so the oracle map is
    # the per-pixel 3x3 solve
    b = _b()
    P = _mixed_problem(synth.C1_BINNED)
    assert P.t_psi.dtype == torch.float32
    out = b.Solver(P.pt, P.nz, tol=1e-10, mixed=1).solve(P.t_d)
    info = out["info"]
    assert info["converged"] == 1 and info["true_rel_resid"] <= 1e-10
    x = out["x"].cpu().numpy()
    x_ref = oracle.binned_map(P.opt, P.d)
    err = oracle.rel_l2_per_stokes(x, x_ref)
    assert np.all(err < 1e-10), err


def test_precision_form_toeplitz_refined():
    b = _b()
    P = _mixed_problem(RAGGED)
    P.pt.attach_weights()
    # FP32 operator alone (one outer step, inner solve run to FP32 accuracy),
    # from x = 0 and from the block-Jacobi map M b (whose residual is FP64)
    _, _, x_ref = oracle.solve(P.opt, P.noise, P.d, tol=1e-14)
    errs = {}
    for bj in (0, 1):
        one = b.Solver(P.pt, P.nz, tol=1e-14, mixed=1, max_outer=1, inner_tol=1e-9, max_iter=400,
                       bj_start=bj).solve(P.t_d)
        errs[bj] = oracle.rel_l2_per_stokes(one["x"].cpu().numpy(), x_ref)
    # FP32 rounding of the I-dominated timeline (sigma_I = 100 vs 1 for Q, U)
    # and of the FP32 (cos 2psi, sin 2psi) leaks ~eps_32 * 100 into Q/U
    print("FP32-operator map error before refinement (I, Q, U): from 0", errs[0], "from M b", errs[1])
    assert np.all(errs[0] < 1e-3) and np.all(errs[1] < 1e-3)
    # refined to a tight FP64 residual: the map matches the FP64 oracle
    out = b.Solver(P.pt, P.nz, tol=1e-13, mixed=1, max_outer=20).solve(P.t_d, history=True)
    info = out["info"]
    assert info["converged"] == 1 and info["true_rel_resid"] <= 1e-13
    assert info["outer_iters"] >= 2
    err = oracle.rel_l2_per_stokes(out["x"].cpu().numpy(), x_ref)
    print("refined map error (I, Q, U):", err, "outer steps", info["outer_iters"], "inner iters", info["iters"])
    assert np.all(err < 1e-10), err
    # FP64 residual history decreases monotonically across outer steps
    h = out["history"]
    assert np.all(np.diff(h) < 0)


# a sparse, wide scan: 8 detectors x 2^20 samples on a 1024^2 grid; a tile's
# pixel window is wider than the LDS bins, so P^T bins it in several passes
WIDE = synth.Workload("wide_1024x1024_8x2^20", 941, 1024, 1024, 8, 1 << 20, t_psi=1500.0, noise="oneoverf",
                      chunk=1 << 18, lam=256)


def test_fused_toeplitz_wide_window_matches_oracle():
    b = _b()
    P = Problem(WIDE, with_d=True).device()
    o = P.opt
    # the valid part of one FP64 tile (2^14 - 2*255 samples) spans more
    # compact indices than the 5760 LDS bins, so several passes are taken
    k = o.compact[P.pix[:(1 << 14) - 510]]
    k = k[k >= 0]
    assert k.max() - k.min() + 1 > 5760
    assert 0.05 < o.mask.mean() < 0.6  # a realistic masked fraction
    P.pt.attach_weights()
    x = np.random.default_rng(21).normal(size=3 * o.n_kept)
    tx = torch.from_numpy(x).to(DEV)
    q_ref = oracle.apply_A(o, P.noise, x)
    # plain tiles (0), and halo-carrying segments (4, 5): 2^23 samples in 8192-
    # sample carry strides make 1024 carrying tiles, i.e. segments of 4 tiles
    # on 256 CUs, so the carried P x and index ranges are exercised, with
    # several bin passes per tile
    for v in (0, 4, 5, 8, 9, 16):
        assert rel_err(b.apply_A(P.pt, P.nz, tx, variant=v).cpu().numpy(), q_ref, 3) < 1e-12, v
        # FP32 timeline arithmetic (32768-sample tiles, more passes): FP32 rounding only
        assert rel_err(b.apply_A(P.pt, P.nz, tx, arith="f32", variant=v).cpu().numpy(), q_ref, 3) < 1e-5, v
    bb = b.rhs(P.pt, P.nz, P.t_d).cpu().numpy()
    assert rel_err(bb, oracle.rhs(o, P.noise, P.d), 3) < 1e-12
