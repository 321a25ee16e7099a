"""Degenerate inputs on the GPU: every pixel masked (no unknowns), and
template intervals of length zero and one."""
import numpy as np
import pytest

import oracle.mapmaking as oracle
from paper_2501_16122_amd import synth
from parity_util import err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"
W = synth.Workload("edges_32x32_2x20000", 961, 32, 32, 2, 20000, t_psi=300.0, noise="oneoverf", chunk=7000, lam=300)


def _b():
    from paper_2501_16122_amd import binding
    return binding


@pytest.mark.parametrize("stokes", ["IQU", "I"])
def test_every_pixel_masked(stokes):
    b = _b()
    pix, psi = synth.pointing(W)
    offs, wdet = synth.det_offsets(W), synth.det_weight(W)
    pt = b.Pointing(torch.from_numpy(pix).to(DEV), torch.from_numpy(psi).to(DEV), offs, wdet, W.n_pix,
                    min_hits=10 ** 6, stokes=stokes)
    assert pt.n_kept == 0
    pt.attach_weights()
    d = torch.from_numpy(np.random.default_rng(1).normal(size=W.n_samples)).to(DEV)
    x = torch.empty(0, dtype=torch.float64, device=DEV)
    for nz in (b.Noise.white(wdet, DEV), b.Noise.toeplitz(synth.toeplitz_coeff(W), synth.chunk_offsets(W), DEV),
               b.Noise.templates(wdet, np.array([0, 5000, W.n_samp, W.n_samples]), 2, DEV)):
        assert b.apply_A(pt, nz, x).numel() == 0
        assert b.rhs(pt, nz, d).numel() == 0
        assert torch.count_nonzero(b.apply_P(pt, x)) == 0
        out = b.Solver(pt, nz).solve(d)
        assert out["info"]["converged"] == 1 and torch.count_nonzero(out["map"]) == 0
    torch.cuda.synchronize()


def test_empty_and_single_sample_intervals():
    b = _b()
    pix, psi = synth.pointing(W)
    offs, wdet = synth.det_offsets(W), synth.det_weight(W)
    opt = oracle.build_pointing(pix, psi, offs, wdet, W.n_pix)
    pt = b.Pointing(torch.from_numpy(pix).to(DEV), torch.from_numpy(psi).to(DEV), offs, wdet, W.n_pix)
    ivals = np.array([0, 0, 1, 1, 2, 700, W.n_samp, W.n_samp, W.n_samp + 1, W.n_samples])
    nz = b.Noise.templates(wdet, ivals, 3, DEV)
    ref_noise = oracle.template_noise(ivals, 3)
    x = np.random.default_rng(2).normal(size=3 * opt.n_kept)
    q = b.apply_A(pt, nz, torch.from_numpy(x).to(DEV)).cpu().numpy()
    ref = oracle.apply_A(opt, ref_noise, x)
    assert err(q, ref, 3) <= 1e-12
    y = np.random.default_rng(3).normal(size=W.n_samples)
    z = b.apply_Ninv(nz, pt, torch.from_numpy(y).to(DEV)).cpu().numpy()
    zr = oracle.apply_w_templates(opt, ref_noise, y)
    assert err(z, zr) <= 1e-12
    # a one-sample interval with any order keeps nothing of that sample
    assert z[0] == 0.0 and abs(z[W.n_samp]) < 1e-15
