"""The allocation-free solve (mm_solve_noalloc) through the C ABI against
the workspace solve (mm_solve) of the same problems: two calls in a row, the
second on a smaller problem, so state left by the first call must not leak
into the second; FP64 at a fixed iteration count and mixed precision to a
tolerance.  Also: a problem larger than the scratch array is refused before
any work."""
import ctypes

import numpy as np
import pytest

import oracle.mapmaking as oracle
from paper_2501_16122_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"

BIG = synth.Workload("noalloc_128x128_3x2^17_toeplitz512", 971, 128, 128, 3, 1 << 17, t_psi=1500.0,
                     noise="oneoverf", chunk=(1 << 15) + 99, lam=512)
SMALL = synth.Workload("noalloc_48x48_2x40000_toeplitz128", 972, 48, 48, 2, 40000, t_psi=900.0,
                       noise="oneoverf", chunk=16384, lam=128)


def _b():
    from paper_2501_16122_amd import binding
    return binding


def _problem(w, precision="f64"):
    b = _b()
    w = w.replace(precision=precision)
    pix, psi = synth.pointing(w)
    psi = synth.storage(w, psi)
    offs, wdet = synth.det_offsets(w), synth.det_weight(w)
    opt = oracle.build_pointing(pix, psi, offs, wdet, w.n_pix)
    d = synth.storage(w, oracle.apply_P(opt, synth.sky(w)[opt.kept].reshape(-1)) + synth.noise(w))
    pt = b.Pointing(torch.from_numpy(pix).to(DEV), torch.from_numpy(psi).to(DEV), offs, wdet, w.n_pix)
    pt.attach_weights()
    nz = b.Noise.toeplitz(synth.toeplitz_coeff(w), synth.chunk_offsets(w), DEV)
    return pt, nz, torch.from_numpy(d).to(DEV), opt


def _noalloc(pt, nz, tod, **opts):
    b = _b()
    o = b.solve_opts(**opts)
    info = b.SolveInfo()
    x = torch.empty(pt.ncomp * pt.n_kept, dtype=torch.float64, device=DEV)
    m = torch.empty(pt.ncomp * pt.n_pix, dtype=torch.float64, device=DEV)
    rc = b.load().mm_solve_noalloc(pt.handle, nz.handle, tod.data_ptr(), m.data_ptr(), x.data_ptr(),
                                   ctypes.byref(o), ctypes.byref(info), torch.cuda.current_stream().cuda_stream)
    return rc, x, m, info.as_dict()


@pytest.mark.parametrize("mixed", [0, 1])
def test_noalloc_matches_workspace_solve_two_calls(mixed):
    b = _b()
    opts = dict(fixed_iter=20, tol=0.0) if not mixed else dict(tol=1e-10, mixed=1, max_outer=20)
    prec = "f32" if mixed else "f64"
    for w in (BIG, SMALL):  # the second call is smaller than the first
        pt, nz, tod, opt = _problem(w, prec)
        ref = b.Solver(pt, nz, **opts).solve(tod)
        rc, x, m, info = _noalloc(pt, nz, tod, **opts)
        assert rc == b.MM_OK, (w.name, rc, b.load().mm_last_error())
        assert info["iters"] == ref["info"]["iters"], (info, ref["info"])
        assert info["converged"] == ref["info"]["converged"]
        err = oracle.rel_l2_per_stokes(x.cpu().numpy(), ref["x"].cpu().numpy())
        assert np.all(err < 1e-10), (w.name, err)
        full = m.cpu().numpy().reshape(-1, 3)
        assert np.all(full[opt.mask] == 0)
        assert np.array_equal(full[opt.kept], x.cpu().numpy().reshape(-1, 3))
        if not mixed:  # and against the oracle's iterate after the same 20 iterations
            _, _, x_ref = oracle.solve(opt, oracle.toeplitz_noise(synth.toeplitz_coeff(w), synth.chunk_offsets(w)),
                                       torch.as_tensor(tod).cpu().numpy(), fixed_iters=20)
            assert np.all(oracle.rel_l2_per_stokes(x.cpu().numpy(), x_ref) < 1e-10)
        pt.close()
        nz.close()


def test_noalloc_refuses_what_it_cannot_hold():
    b = _b()
    # a 1024^2 I, Q, U map with every pixel kept: ~3.1 million unknowns of
    # solver state, more than the scratch array holds: refused before work
    w = synth.Workload("noalloc_1024x1024_6x2^20", 973, 1024, 1024, 6, 1 << 20, t_psi=900.0, noise="oneoverf",
                       chunk=1 << 15, lam=64)
    t = np.arange(w.n_samples, dtype=np.int64)
    pix = (t // 6).astype(np.int32)           # six consecutive samples per pixel
    psi = (t % 6) * (np.pi / 6)               # at equispaced 2 psi: cond = 2, kept
    offs, wdet = synth.det_offsets(w), synth.det_weight(w)
    pt = b.Pointing(torch.from_numpy(pix).to(DEV), torch.from_numpy(psi).to(DEV), offs, wdet, w.n_pix)
    assert pt.n_kept == w.n_pix
    nz = b.Noise.toeplitz(synth.toeplitz_coeff(w), synth.chunk_offsets(w), DEV)
    tod = torch.zeros(w.n_samples, dtype=torch.float64, device=DEV)
    rc, _, _, _ = _noalloc(pt, nz, tod, fixed_iter=2, tol=0.0)
    assert rc == b.MM_ENOSPC
    assert b"scratch" in b.load().mm_last_error()
    pt.close()
    nz.close()
    # options that would allocate events or graphs are refused
    pt2, nz2, tod2, _ = _problem(SMALL)
    for bad in (dict(autotune=1), dict(timing=1), dict(graph=1)):
        rc, _, _, _ = _noalloc(pt2, nz2, tod2, **bad)
        assert rc == b.MM_EINVAL, bad
