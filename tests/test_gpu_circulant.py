"""Circulant N^-1 per stationary chunk (the band filter on each chunk taken
as periodic) on the GPU against the oracle: the weighting alone, the fused
operator in every variant, the right-hand side and the solve."""
import numpy as np
import pytest

import oracle.mapmaking as oracle
from paper_2501_16122_amd import synth
from parity_util import err as rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"

# ragged chunks: 3 detectors of 3*2^16 + 777 samples, chunks of 2^15 + 123
W = synth.Workload("circ_128x128_3x197385", 951, 128, 128, 3, 3 * (1 << 16) + 777, t_psi=1500.0,
                   noise="oneoverf", chunk=(1 << 15) + 123, lam=512)


def circ_chunks(w):
    """The workload's chunks, with a chunk shorter than the band merged into
    the one before it (a circulant chunk must be longer than 2 (lam - 1))."""
    offs = list(synth.chunk_offsets(w))
    det = set(synth.det_offsets(w).tolist())
    out = [offs[0]]
    for a, b in zip(offs[:-1], offs[1:]):
        if b - a <= 2 * (w.lam - 1) and a not in det:
            out[-1] = b
        else:
            out.append(b)
    return np.array(out, dtype=np.int64)


def _b():
    from paper_2501_16122_amd import binding
    return binding


@pytest.fixture(scope="module")
def prob():
    b = _b()
    pix, psi = synth.pointing(W)
    offs, wdet = synth.det_offsets(W), synth.det_weight(W)
    opt = oracle.build_pointing(pix, psi, offs, wdet, W.n_pix)
    coeff, chunks = synth.toeplitz_coeff(W), circ_chunks(W)
    noise = oracle.circulant_noise(coeff, chunks)
    d = oracle.apply_P(opt, synth.sky(W)[opt.kept].reshape(-1)) + synth.noise(W)
    pt = b.Pointing(torch.from_numpy(pix).to(DEV), torch.from_numpy(psi).to(DEV), offs, wdet, W.n_pix)
    pt.attach_weights()
    nz = b.Noise.circulant(coeff, chunks, DEV)
    return opt, noise, d, pt, nz


@pytest.mark.parametrize("lam", [1, 64, 512, 4096])
def test_circulant_ninv_matches_oracle(prob, lam):
    b = _b()
    opt, _, _, pt, _ = prob
    w = W.replace(lam=lam)
    coeff = synth.toeplitz_coeff(w)
    # the detector-aligned chunks, plus one chunk barely longer than the band
    chunks = circ_chunks(w)
    chunks = np.sort(np.unique(np.concatenate([chunks, [chunks[1] - (2 * lam - 1)]])))
    y = np.random.default_rng(lam).normal(size=W.n_samples)
    z = b.apply_Ninv(b.Noise.circulant(coeff, chunks, DEV), pt, torch.from_numpy(y).to(DEV)).cpu().numpy()
    ref = oracle.apply_ninv_circulant(oracle.circulant_noise(coeff, chunks), y)
    assert rel(z, ref) < 1e-12
    # near the chunk edges the wrap-around differs from the band section
    if lam > 1:
        zt = oracle.apply_ninv_toeplitz(oracle.toeplitz_noise(coeff, chunks), y)
        assert rel(zt, ref) > 1e-6


def test_circulant_fused_operator_all_variants(prob):
    b = _b()
    opt, noise, d, pt, nz = prob
    x = np.random.default_rng(7).normal(size=3 * opt.n_kept)
    ref = oracle.apply_A(opt, noise, x)
    tx = torch.from_numpy(x).to(DEV)
    for v in list(range(8)) + [8, 9, 16, 17]:
        assert rel(b.apply_A(pt, nz, tx, variant=v).cpu().numpy(), ref, 3) < 1e-12, v
        assert rel(b.apply_A(pt, nz, tx, arith="f32", variant=v).cpu().numpy(), ref, 3) < 1e-5, v
    bb = b.rhs(pt, nz, torch.from_numpy(d).to(DEV)).cpu().numpy()
    assert rel(bb, oracle.rhs(opt, noise, d), 3) < 1e-12


def test_circulant_solve_matches_oracle(prob):
    b = _b()
    opt, noise, d, pt, nz = prob
    td = torch.from_numpy(d).to(DEV)
    out = b.Solver(pt, nz, fixed_iter=20, tol=0.0).solve(td)
    _, _, x_ref = oracle.solve(opt, noise, d, fixed_iters=20)
    assert np.all(oracle.rel_l2_per_stokes(out["x"].cpu().numpy(), x_ref) < 1e-10)
    conv = b.Solver(pt, nz, tol=1e-12, autotune=1).solve(td)
    assert conv["info"]["converged"] == 1 and conv["info"]["true_rel_resid"] <= 1e-11


def test_circulant_rejects_short_chunks():
    b = _b()
    coeff = synth.toeplitz_coeff(W.replace(lam=64))
    with pytest.raises(b.MapMakerError):
        b.Noise.circulant(coeff, np.array([0, 100, 226]), DEV)  # 126 <= 2 * 63


def test_circulant_in_batched_steps(prob):
    # a circulant member shares the band-Toeplitz batch launches (its tiles
    # carry the wrap flag) and matches the same solve alone
    b = _b()
    opt, noise, d, pt, nz = prob
    td = torch.from_numpy(d).to(DEV)
    opts = dict(tol=1e-11, check_every=4)
    alone = b.Solver(pt, nz, **opts).solve(td)["x"].cpu().numpy()
    s1 = b.AsyncSolver(pt, nz, td, **opts)
    s2 = b.AsyncSolver(pt, b.Noise.white(synth.det_weight(W), DEV), td, **opts)
    for _ in range(200):
        b.batch_step([s1, s2], 4)
        torch.cuda.synchronize()
        if s1.poll()[0] and s2.poll()[0]:
            break
    r1 = s1.finish()
    assert r1["info"][0]["converged"] == 1
    assert np.all(oracle.rel_l2_per_stokes(r1["x"][0].cpu().numpy(), alone) < 1e-10)
    assert s2.finish()["info"][0]["converged"] == 1
