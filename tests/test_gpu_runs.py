"""P^T on timelines made of long runs of one pixel: the scatter sums runs of
equal pixels across neighbouring lanes before its bin atomics, so runs that
cross wavefront, block and tile boundaries, runs of masked pixels, and ragged
tile tails are checked against the oracle in every map form."""
import numpy as np
import pytest

import oracle.mapmaking as oracle
from parity_util import err as rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"
N_PIX = 40
N_DET, N_SAMP = 3, 50001


def _b():
    from paper_2501_16122_amd import binding
    return binding


def _timeline(seed=11):
    """Runs of 1..400 samples of one pixel (pixels 0..37, random angles);
    pixel 38 is seen twice (too few hits for I, Q, U), pixel 39 fifty times
    at one angle (a singular block where the row uses the angle), both
    inside the runs."""
    rng = np.random.default_rng(seed)
    n = N_DET * N_SAMP
    pix = np.empty(n, dtype=np.int32)
    i = 0
    while i < n:
        ln = int(min(n - i, rng.choice([1, 2, 3, 5, 17, 63, 64, 65, 130, 257, 400])))
        pix[i:i + ln] = rng.integers(0, 38)
        i += ln
    psi = rng.uniform(0.0, np.pi, size=n)
    pix[[1000, 70000]] = 38
    at = np.arange(5000, 5050)
    pix[at] = 39
    psi[at] = 0.3
    offs = np.arange(N_DET + 1, dtype=np.int64) * N_SAMP
    wdet = 1.0 / (1.0 + 0.5 * np.arange(N_DET))
    return pix, psi, offs, wdet


@pytest.mark.parametrize("stokes", ["IQU", "QU", "I"])
def test_pt_on_long_runs(stokes):
    b = _b()
    pix, psi, offs, wdet = _timeline()
    opt = oracle.build_pointing(pix, psi, offs, wdet, N_PIX, stokes=stokes)
    # masked: pixel 38 needs 3 hits for I, Q, U; pixel 39 is singular unless the form has no angle
    expect = {"IQU": [True, True], "QU": [False, True], "I": [False, False]}[stokes]
    assert not opt.mask[:38].any() and list(opt.mask[38:]) == expect
    pt = b.Pointing(torch.from_numpy(pix).to(DEV), torch.from_numpy(psi).to(DEV), offs, wdet, N_PIX, stokes=stokes)
    assert pt.n_kept == opt.n_kept
    y = np.random.default_rng(5).normal(size=pix.size)
    ty = torch.from_numpy(y).to(DEV)
    assert rel(b.apply_PT(pt, ty).cpu(), oracle.apply_PT(opt, y), opt.ncomp) < 1e-13
    # the white right-hand side runs the same scatter with detector weights
    nz = b.Noise.white(wdet, DEV)
    assert rel(b.rhs(pt, nz, ty).cpu(), oracle.rhs(opt, None, y), opt.ncomp) < 1e-13
    # and the adjoint identity <P x, y> = <x, P^T y> on these runs
    x = np.random.default_rng(6).normal(size=opt.ncomp * opt.n_kept)
    px = b.apply_P(pt, torch.from_numpy(x).to(DEV)).cpu().numpy()
    pty = b.apply_PT(pt, ty).cpu().numpy()
    assert abs(px @ y - x @ pty) <= 1e-12 * np.linalg.norm(px) * np.linalg.norm(y)


def test_pt_single_pixel_timeline():
    # one pixel for the whole timeline: every wavefront is one run
    b = _b()
    rng = np.random.default_rng(8)
    n = 2 * 40000 + 3
    pix = np.zeros(n, dtype=np.int32)
    psi = rng.uniform(0.0, np.pi, size=n)
    offs = np.array([0, 40000, n], dtype=np.int64)
    wdet = np.array([1.0, 2.0])
    opt = oracle.build_pointing(pix, psi, offs, wdet, 1)
    pt = b.Pointing(torch.from_numpy(pix).to(DEV), torch.from_numpy(psi).to(DEV), offs, wdet, 1)
    y = rng.normal(size=n)
    assert rel(b.apply_PT(pt, torch.from_numpy(y).to(DEV)).cpu(), oracle.apply_PT(opt, y), 3) < 1e-12
