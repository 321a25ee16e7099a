"""Polarisation-only (QU) and intensity-only (I) map forms on the GPU against
the oracle: the build (bit-exact integers), every operator (white and
band-Toeplitz, all fused-operator variants, FP64 and FP32 timeline
arithmetic), the solve at a fixed iteration count, the mixed-precision solve
and batched steps.  Same bar as the I, Q, U form."""
import numpy as np
import pytest

import oracle.mapmaking as oracle
from paper_2501_16122_amd import synth
from parity_util import err as rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"

# several pointing and FFT tiles with ragged tails on a 128^2 grid
W = synth.Workload("forms_128x128_3x197385", 941, 128, 128, 3, 3 * (1 << 16) + 777, t_psi=1500.0,
                   noise="oneoverf", chunk=(1 << 15) + 123, lam=512)
FORMS = ["QU", "I"]


def _b():
    from paper_2501_16122_amd import binding
    return binding


class Form:
    def __init__(self, stokes, precision="f64", psi_none=False):
        b = _b()
        w = W.replace(precision=precision)
        pix, psi = synth.pointing(w)
        self.psi = synth.storage(w, psi)
        self.offs, self.wdet = synth.det_offsets(w), synth.det_weight(w)
        self.opt = oracle.build_pointing(pix, self.psi, self.offs, self.wdet, w.n_pix, stokes=stokes)
        self.nc = self.opt.ncomp
        self.coeff, self.chunks = synth.toeplitz_coeff(w), synth.chunk_offsets(w)
        self.noise = oracle.toeplitz_noise(self.coeff, self.chunks)
        m = np.random.default_rng(3).normal(size=self.nc * self.opt.n_kept) * 5.0
        self.d = synth.storage(w, oracle.apply_P(self.opt, m) + synth.noise(w))
        self.t_pix = torch.from_numpy(pix).to(DEV)
        self.t_psi = None if psi_none else torch.from_numpy(self.psi).to(DEV)
        tdt = torch.float64 if precision == "f64" else torch.float32
        self.pt = b.Pointing(self.t_pix, self.t_psi, self.offs, self.wdet, w.n_pix, stokes=stokes, tod_dtype=tdt)
        self.pt.attach_weights()
        self.nz = b.Noise.toeplitz(self.coeff, self.chunks, DEV)
        self.white = b.Noise.white(self.wdet, DEV)
        self.t_d = torch.from_numpy(self.d).to(DEV)


@pytest.fixture(scope="module", params=FORMS)
def form(request):
    return Form(request.param)


def test_build_bit_exact(form):
    o, pt = form.opt, form.pt
    ex = pt.export()
    assert pt.n_kept == o.n_kept and pt.ncomp == form.nc
    assert np.array_equal(ex["hits"].cpu().numpy(), o.hits.astype(np.int32))
    assert np.array_equal(ex["mask"].cpu().numpy().astype(bool), o.mask)
    assert np.array_equal(ex["compact"].cpu().numpy(), o.compact.astype(np.int32))
    assert np.array_equal(ex["kept"].cpu().numpy(), o.kept.astype(np.int32))
    assert rel(ex["minv"].cpu().numpy(), o.minv, form.nc ** 2) < 1e-12
    assert oracle.mask_margin(o) > 1e-9
    # the forms mask differently: I keeps every seen pixel
    if form.nc == 1:
        assert o.n_kept == int(np.count_nonzero(o.hits))


def test_intensity_form_reads_no_angle():
    b = _b()
    f = Form("I", psi_none=True)
    g = Form("I")
    assert np.array_equal(f.pt.export()["kept"].cpu().numpy(), g.pt.export()["kept"].cpu().numpy())
    x = torch.from_numpy(np.random.default_rng(1).normal(size=f.opt.n_kept)).to(DEV)
    assert torch.equal(b.apply_A(f.pt, f.nz, x), b.apply_A(g.pt, g.nz, x)) or \
        rel(b.apply_A(f.pt, f.nz, x).cpu(), b.apply_A(g.pt, g.nz, x).cpu()) < 1e-13
    with pytest.raises(ValueError):
        b.Pointing(f.t_pix, None, f.offs, f.wdet, W.n_pix, stokes="QU")


def test_pointing_operators(form):
    b = _b()
    o = form.opt
    rng = np.random.default_rng(2)
    x = rng.normal(size=form.nc * o.n_kept)
    y = rng.normal(size=o.n_samples)
    tx, ty = torch.from_numpy(x).to(DEV), torch.from_numpy(y).to(DEV)
    assert rel(b.apply_P(form.pt, tx).cpu(), oracle.apply_P(o, x)) < 1e-14
    assert rel(b.apply_PT(form.pt, ty).cpu(), oracle.apply_PT(o, y), form.nc) < 1e-13
    assert rel(b.apply_M(form.pt, tx).cpu(), oracle.apply_M(o, x), form.nc) < 1e-13
    full = b.expand_map(form.pt, tx).cpu().numpy().reshape(-1, form.nc)
    assert np.array_equal(full, oracle.expand(o, x))


def test_fused_operators_all_variants(form):
    b = _b()
    o = form.opt
    x = np.random.default_rng(4).normal(size=form.nc * o.n_kept)
    tx = torch.from_numpy(x).to(DEV)
    ref_w = oracle.apply_A(o, None, x)
    assert rel(b.apply_A(form.pt, form.white, tx).cpu(), ref_w, form.nc) < 1e-13
    assert rel(b.apply_A(form.pt, form.white, tx, arith="f32").cpu(), ref_w, form.nc) < 1e-5
    ref = oracle.apply_A(o, form.noise, x)
    for v in list(range(8)) + [8, 9, 16, 17]:
        assert rel(b.apply_A(form.pt, form.nz, tx, variant=v).cpu(), ref, form.nc) < 1e-12, v
        assert rel(b.apply_A(form.pt, form.nz, tx, arith="f32", variant=v).cpu(), ref, form.nc) < 1e-5, v
    X = torch.stack([tx, 2.0 * tx]).contiguous()
    Q = b.apply_A_multi(form.pt, form.nz, X).cpu().numpy()
    assert rel(Q[0], ref, form.nc) < 1e-12 and rel(Q[1], 2.0 * ref, form.nc) < 1e-12
    assert rel(b.rhs(form.pt, form.nz, form.t_d).cpu(), oracle.rhs(o, form.noise, form.d), form.nc) < 1e-12
    assert rel(b.rhs(form.pt, form.white, form.t_d).cpu(), oracle.rhs(o, None, form.d), form.nc) < 1e-13


def test_white_solve_is_binned_map(form):
    b = _b()
    out = b.Solver(form.pt, form.white, tol=1e-12).solve(form.t_d)
    assert out["info"]["iters"] == 1
    x = out["x"].cpu().numpy()
    assert np.all(oracle.rel_l2_per_stokes(x, oracle.binned_map(form.opt, form.d), ncomp=form.nc) < 1e-12)
    m = out["map"].cpu().numpy().reshape(-1, form.nc)
    assert np.all(m[form.opt.mask] == 0)


def test_toeplitz_solve_fixed_iterations(form):
    b = _b()
    k = 25
    out = b.Solver(form.pt, form.nz, fixed_iter=k, tol=0.0).solve(form.t_d)
    _, info, x_ref = oracle.solve(form.opt, form.noise, form.d, fixed_iters=k)
    assert out["info"]["iters"] == k
    err = oracle.rel_l2_per_stokes(out["x"].cpu().numpy(), x_ref, ncomp=form.nc)
    assert np.all(err < 1e-10), err


def test_mixed_precision_solve(form):
    b = _b()
    f = Form(form.opt.stokes, precision="f32")
    out = b.Solver(f.pt, f.nz, tol=1e-13, mixed=1, max_outer=20, autotune=1).solve(f.t_d)
    assert out["info"]["converged"] == 1 and out["info"]["true_rel_resid"] <= 1e-13
    _, info, x_ref = oracle.solve(f.opt, f.noise, f.d, tol=1e-13)
    # both solved to 1e-13: each map is within about kappa * 1e-13 of the exact one
    err = oracle.rel_l2_per_stokes(out["x"].cpu().numpy(), x_ref, ncomp=f.nc)
    assert np.all(err < 1e-10), err


def test_batched_steps_match_alone(form):
    b = _b()
    opts = dict(tol=1e-11, check_every=4)
    alone = b.Solver(form.pt, form.nz, **opts).solve(form.t_d)["x"].cpu().numpy()
    s1 = b.AsyncSolver(form.pt, form.nz, form.t_d, **opts)
    s2 = b.AsyncSolver(form.pt, form.white, form.t_d, **opts)
    for _ in range(200):
        b.batch_step([s1, s2], 4)
        torch.cuda.synchronize()
        if s1.poll()[0] and s2.poll()[0]:
            break
    r1, r2 = s1.finish(), s2.finish()
    assert r1["info"][0]["converged"] == 1 and r2["info"][0]["converged"] == 1
    assert np.all(oracle.rel_l2_per_stokes(r1["x"][0].cpu().numpy(), alone, ncomp=form.nc) < 1e-10)
    binned = oracle.binned_map(form.opt, form.d)
    assert np.all(oracle.rel_l2_per_stokes(r2["x"][0].cpu().numpy(), binned, ncomp=form.nc) < 1e-10)
