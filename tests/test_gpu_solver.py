"""Resumable and multi-right-hand-side solves, and the continuous-batching
server: each result equals the same problem solved alone, and the oracle."""
import numpy as np
import pytest

import oracle.mapmaking as oracle
from paper_2501_16122_amd import synth
from parity_util import err as op_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"


def _b():
    from paper_2501_16122_amd import binding
    return binding


SMALL_T = synth.Workload("small_toeplitz_64x64_2x60000", 961, 64, 64, 2, 60000, t_psi=900.0, noise="oneoverf",
                         chunk=20000, lam=256)


def _device_problem(w, n_rhs=1):
    b = _b()
    pix, psi = synth.pointing(w)
    psi = synth.storage(w, psi)
    offs, wdet = synth.det_offsets(w), synth.det_weight(w)
    opt = oracle.build_pointing(pix, psi, offs, wdet, w.n_pix)
    noise = oracle.toeplitz_noise(synth.toeplitz_coeff(w), synth.chunk_offsets(w)) if w.toeplitz else None
    m = synth.sky(w)[opt.kept].reshape(-1)
    ds = []
    for r in range(n_rhs):
        wr = w.replace(config_id=w.config_id * 100 + r)  # one noise realisation per right-hand side
        ds.append(synth.storage(w, oracle.apply_P(opt, m) + synth.noise(wr)))
    pt = b.Pointing(torch.from_numpy(pix).to(DEV), torch.from_numpy(psi).to(DEV), offs, wdet, w.n_pix)
    nz = (b.Noise.toeplitz(synth.toeplitz_coeff(w), synth.chunk_offsets(w), DEV) if w.toeplitz
          else b.Noise.white(wdet, DEV))
    return pt, nz, opt, noise, ds


def test_async_solver_matches_blocking_solve():
    b = _b()
    pt, nz, opt, noise, ds = _device_problem(SMALL_T)
    td = torch.from_numpy(ds[0]).to(DEV)
    ref = b.Solver(pt, nz, tol=1e-10).solve(td)
    s = b.AsyncSolver(pt, nz, td, tol=1e-10, check_every=4)
    steps = 0
    while True:
        s.step()
        s.stream.synchronize()
        done, in_flight = s.poll()
        assert not in_flight
        steps += 1
        if done:
            break
        assert steps < 1000
    out = s.finish()
    assert out["info"][0]["iters"] == ref["info"]["iters"]
    err = oracle.rel_l2_per_stokes(out["x"][0].cpu().numpy(), ref["x"].cpu().numpy())
    assert np.all(err < 1e-12), err


def test_apply_A_multi_matches_single():
    b = _b()
    pt, nz, opt, noise, ds = _device_problem(SMALL_T)
    pt.attach_weights()
    X = torch.randn(5, 3 * pt.n_kept, dtype=torch.float64, device=DEV)
    Q = b.apply_A_multi(pt, nz, X)
    for r in range(5):
        q = b.apply_A(pt, nz, X[r].contiguous())
        assert op_err(Q[r], q, 3) < 1e-13
    # and against the oracle
    q0 = oracle.apply_A(opt, noise, X[2].cpu().numpy())
    assert op_err(Q[2], q0, 3) < 1e-12


@pytest.mark.parametrize("mixed", [0, 1])
def test_multi_rhs_solve_equals_single_solves(mixed):
    b = _b()
    w = SMALL_T if not mixed else SMALL_T.replace(precision="f32")
    pt, nz, opt, noise, ds = _device_problem(w, n_rhs=4)
    pt.attach_weights()
    tods = torch.from_numpy(np.stack(ds)).to(DEV)
    # solved to 1e-13, so that the map is within about kappa * 1e-13 of the
    # exact one and the oracle comparison below can use 1e-10
    multi = b.AsyncSolver(pt, nz, tods, tol=1e-13, mixed=mixed, max_outer=20)
    while True:
        multi.step()
        multi.stream.synchronize()
        done, _ = multi.poll()
        if done:
            break
    out = multi.finish()
    for r in range(4):
        single = b.Solver(pt, nz, tol=1e-13, mixed=mixed, max_outer=20).solve(tods[r].contiguous())
        err = oracle.rel_l2_per_stokes(out["x"][r].cpu().numpy(), single["x"].cpu().numpy())
        assert np.all(err < 1e-10), (r, err)
        assert out["info"][r]["converged"] == 1
    # one right-hand side against the oracle on the same (rounded) inputs
    _, _, x_ref = oracle.solve(opt, noise, ds[1].astype(np.float64), tol=1e-13)
    err = oracle.rel_l2_per_stokes(out["x"][1].cpu().numpy(), x_ref)
    assert np.all(err < 1e-10), err


def _serving_requests():
    from paper_2501_16122_amd import serve

    def sizes(rng, i):
        side = serve.log_uniform_int(rng, 32, 96)
        n_det = serve.log_uniform_int(rng, 1, 4)
        n_samp = serve.log_uniform_int(rng, 20000, 120000)
        toep = rng.uniform() < 0.5
        return synth.Workload(f"serve_{i}", 970 + i, side, side, n_det, n_samp, t_psi=700.0,
                              noise="oneoverf" if toep else "white", chunk=32768 if toep else 0,
                              lam=512 if toep else 0, precision="f32")

    reqs = serve.poisson_requests(7, 200.0, sizes, seed_id=77)

    def make_d(w, pix, psi):
        opt = oracle.build_pointing(pix, psi, synth.det_offsets(w), synth.det_weight(w), w.n_pix)
        return oracle.apply_P(opt, synth.sky(w)[opt.kept].reshape(-1)) + synth.noise(w)

    return [serve.materialize(r, make_d) for r in reqs], make_d


def test_serving_mix_equals_alone():
    from paper_2501_16122_amd import serve
    reqs, _ = _serving_requests()
    # alone: one slot, one request at a time.  Solved to a 1e-12 residual:
    # runs stopped at 1e-10 may sit at different iterates (FP64 atomics
    # reorder sums), and a 1e-10 residual only bounds the map to ~1e-8.
    alone = {r.rid: r for r in serve.Server(DEV, max_slots=1, k_chunk=8, tol=1e-12, max_outer=20).run(
        reqs, realtime=False)}
    reqs2, _ = _serving_requests()
    srv = serve.Server(DEV, max_slots=8, k_chunk=8, tol=1e-12, max_outer=20)
    mix = {r.rid: r for r in srv.run(reqs2, realtime=False)}
    assert srv.peak_slots >= 2, "requests must overlap on the device"
    assert sorted(alone) == sorted(mix) == list(range(7))
    for rid in alone:
        a, m = alone[rid], mix[rid]
        assert a.info["converged"] == 1 and m.info["converged"] == 1
        assert m.info["true_rel_resid"] <= 1e-12
        mask = np.any(a.map != 0, axis=1)
        err = oracle.rel_l2_per_stokes(m.map[mask], a.map[mask])
        assert np.all(err < 1e-10), (rid, err)
    # two requests against the oracle (same rounded inputs)
    for r in reqs2[:2]:
        w = r.workload
        opt = oracle.build_pointing(r.pix, r.psi, synth.det_offsets(w), synth.det_weight(w), w.n_pix)
        nz = oracle.toeplitz_noise(r.coeff, r.chunks) if w.toeplitz else None
        m_ref, _, _ = oracle.solve(opt, nz, r.d.astype(np.float64), tol=1e-13)
        err = oracle.rel_l2_per_stokes(mix[r.rid].map[opt.kept], m_ref[opt.kept])
        assert np.all(err < 1e-9), (r.rid, err)


def test_batched_serving_mix_equals_alone():
    """The batched server (one shared step for all active solves) gives each
    request the result it gets alone."""
    from paper_2501_16122_amd import serve
    reqs, _ = _serving_requests()
    alone = {r.rid: r for r in serve.Server(DEV, max_slots=1, k_chunk=8, tol=1e-12, max_outer=20).run(
        reqs, realtime=False)}
    reqs2, _ = _serving_requests()
    srv = serve.Server(DEV, max_slots=8, k_chunk=8, tol=1e-12, max_outer=20, batched=True)
    mix = {r.rid: r for r in srv.run(reqs2, realtime=False)}
    assert srv.peak_slots >= 2
    assert sorted(alone) == sorted(mix) == list(range(7))
    for rid in alone:
        a, m = alone[rid], mix[rid]
        assert m.info["converged"] == 1 and m.info["true_rel_resid"] <= 1e-12
        mask = np.any(a.map != 0, axis=1)
        err = oracle.rel_l2_per_stokes(m.map[mask], a.map[mask])
        assert np.all(err < 1e-10), (rid, err)
    with pytest.raises(ValueError):
        serve.Server(DEV, max_slots=17, batched=True)


@pytest.mark.parametrize("batched", [False, True])
def test_serving_cancel_frees_and_keeps_others(batched):
    """A request cancelled while queued and one cancelled while active (its
    chunks of iterations still in flight) are withdrawn: their device memory
    is freed, and every other request still converges."""
    import gc
    import torch
    from paper_2501_16122_amd import serve
    reqs, _ = _serving_requests()
    torch.cuda.synchronize()
    gc.collect()
    before = torch.cuda.memory_allocated(DEV)
    srv = serve.Server(DEV, max_slots=3, k_chunk=8, tol=1e-12, max_outer=20, batched=batched)
    srv.cancel(6)  # still queued when the run starts
    asked = []

    def on_result(res):
        if asked:
            return
        for sl in list(srv.active):
            if sl.req.rid not in (res.rid, 6):
                asked.append(sl.req.rid)
                srv.cancel(sl.req.rid)
                break

    res = srv.run(reqs, realtime=False, on_result=on_result)
    stages = {rid: stage for rid, stage, _ in srv.cancelled}
    print(f"batched={batched}: cancelled {stages}, asked {asked}", flush=True)
    assert stages[6] == "queued"
    assert asked
    # a solve that finished in the tick its cancel arrived is a result
    if asked[0] in stages:
        assert stages[asked[0]] == "active"
    done = {r.rid for r in res}
    assert done | set(stages) == set(range(7)) and not (done & set(stages))
    for r in res:
        assert r.info["converged"] == 1 and r.info["true_rel_resid"] <= 1e-12, r.rid
    assert srv.in_use == 0
    del srv, res
    torch.cuda.synchronize()
    gc.collect()
    assert torch.cuda.memory_allocated(DEV) <= before + (1 << 20)


def test_serving_respects_memory_budget():
    from paper_2501_16122_amd import serve
    reqs, _ = _serving_requests()
    fps = [serve.footprint_bytes(r.workload, _b().solve_opts(mixed=1, tol=1e-10), r.workload.toeplitz)
           for r in reqs]
    budget = int(1.01 * max(fps))  # room for the largest request alone
    assert sum(fps) > budget
    srv = serve.Server(DEV, hbm_budget=budget, max_slots=8)
    res = srv.run(reqs, realtime=False)
    assert len(res) == 7 and all(r.info["converged"] == 1 for r in res)
    assert srv.peak_bytes <= budget
    # everything arrived at t = 0, so memory, not slots, made some wait
    assert srv.peak_slots < 7
    assert max(r.admitted for r in res) > min(r.finished for r in res)


def test_serving_poisson_stream_latencies():
    from paper_2501_16122_amd import serve
    reqs, _ = _serving_requests()
    srv = serve.Server(DEV, max_slots=4, k_chunk=8)
    res = srv.run(reqs, realtime=True)
    assert len(res) == 7 and all(r.info["converged"] == 1 for r in res)
    lat = np.array([r.latency for r in res])
    assert np.all(lat > 0) and np.all(np.array([r.admitted for r in res]) >= np.array([r.arrival for r in res]) - 1e-9)


def test_operator_variants_agree_and_autotune():
    """Every band-Toeplitz operator variant (tile order, map staging, halo
    carrying, two workgroups per CU) gives the same solve; the autotuner
    picks one of them and remembers it."""
    b = _b()
    pt, nz, opt, noise, ds = _device_problem(SMALL_T)
    pt.attach_weights()
    td = torch.from_numpy(ds[0]).to(DEV)
    ref = b.Solver(pt, nz, tol=1e-12).solve(td)
    for v in list(range(8)) + [8, 9, 16, 17]:
        out = b.Solver(pt, nz, tol=1e-12, op_variant=v).solve(td)
        assert out["info"]["op_variant"] == v
        err = oracle.rel_l2_per_stokes(out["x"].cpu().numpy(), ref["x"].cpu().numpy())
        assert np.all(err < 1e-10), (v, err)
    tuned = b.Solver(pt, nz, tol=1e-12, autotune=1).solve(td)
    assert 0 <= tuned["info"]["op_variant"] < 32
    err = oracle.rel_l2_per_stokes(tuned["x"].cpu().numpy(), ref["x"].cpu().numpy())
    assert np.all(err < 1e-10), err
    again = b.Solver(pt, nz, tol=1e-12, autotune=1).solve(td)  # remembered by the noise handle
    assert again["info"]["op_variant"] == tuned["info"]["op_variant"]
    with pytest.raises(b.MapMakerError):
        b.Solver(pt, nz, op_variant=32).solve(td)
    # the FP32 inner operator with refinement, tuned
    w32 = SMALL_T.replace(precision="f32")
    pt32, nz32, opt32, noise32, ds32 = _device_problem(w32)
    pt32.attach_weights()
    out = b.Solver(pt32, nz32, tol=1e-12, mixed=1, max_outer=20, autotune=1).solve(
        torch.from_numpy(ds32[0]).to(DEV))
    assert out["info"]["converged"] == 1 and 0 <= out["info"]["op_variant"] < 32
    _, _, x_ref = oracle.solve(opt32, noise32, ds32[0].astype(np.float64), tol=1e-13)
    err = oracle.rel_l2_per_stokes(out["x"].cpu().numpy(), x_ref)
    assert np.all(err < 1e-9), err


# long chunks at the largest band: several halo-carrying tiles per segment
LONG4096 = synth.Workload("long_128x128_2x2^18_lam4096", 962, 128, 128, 2, 1 << 18, t_psi=1100.0,
                          noise="oneoverf", chunk=(1 << 17) + 777, lam=4096)


@pytest.mark.parametrize("variant", list(range(8)) + [8, 9, 16])
@pytest.mark.parametrize("w", [SMALL_T, LONG4096], ids=["small", "long4096"])
def test_operator_variants_fixed_iteration_parity(w, variant):
    """Each operator variant, through a fixed number of PCG iterations,
    against the oracle's iterate (FP64)."""
    b = _b()
    pt, nz, opt, noise, ds = _device_problem(w)
    pt.attach_weights()
    out = b.Solver(pt, nz, fixed_iter=15, tol=0.0, op_variant=variant).solve(torch.from_numpy(ds[0]).to(DEV))
    assert out["info"]["iters"] == 15 and out["info"]["op_variant"] == variant
    _, _, x_ref = oracle.solve(opt, noise, ds[0].astype(np.float64), fixed_iters=15)
    err = oracle.rel_l2_per_stokes(out["x"].cpu().numpy(), x_ref)
    assert np.all(err < 1e-10), err


def test_carry_variant_mixed_precision():
    b = _b()
    w = LONG4096.replace(precision="f32")
    pt, nz, opt, noise, ds = _device_problem(w)
    pt.attach_weights()
    out = b.Solver(pt, nz, tol=1e-13, mixed=1, max_outer=20, op_variant=5).solve(torch.from_numpy(ds[0]).to(DEV))
    assert out["info"]["converged"] == 1
    _, _, x_ref = oracle.solve(opt, noise, ds[0].astype(np.float64), tol=1e-13)
    err = oracle.rel_l2_per_stokes(out["x"].cpu().numpy(), x_ref)
    assert np.all(err < 1e-10), err


@pytest.mark.parametrize("white", [False, True])
def test_start_vector_matches_oracle(white):
    # PCG from a start vector x0: the same iterates as the oracle's from x0;
    # started at the solution the solve stops at once; the mixed form refines
    # from x0; several right-hand sides each start from their own x0
    b = _b()
    w = SMALL_T.replace(noise="white", chunk=0, lam=0) if white else SMALL_T
    pt, nz, opt, noise, ds = _device_problem(w, n_rhs=2)
    td = torch.from_numpy(ds[0]).to(DEV)
    rng = np.random.default_rng(31)
    x0 = rng.normal(size=3 * opt.n_kept)
    tx0 = torch.from_numpy(x0).to(DEV)
    k = 1 if white else 12  # white: M = A^-1, one iteration reaches the solution
    out = b.Solver(pt, nz, fixed_iter=k, tol=0.0).solve(td, x0=tx0)
    bb = oracle.rhs(opt, noise, ds[0])
    x_ref, info = oracle.pcg(lambda v: oracle.apply_A(opt, noise, v), lambda v: oracle.apply_M(opt, v), bb,
                             fixed_iters=k, x0=x0)
    assert np.all(oracle.rel_l2_per_stokes(out["x"].cpu().numpy(), x_ref) < 1e-10)
    conv = b.Solver(pt, nz, tol=1e-13).solve(td)
    again = b.Solver(pt, nz, tol=1e-10).solve(td, x0=conv["x"].clone())
    assert again["info"]["iters"] == 0 and again["info"]["converged"] == 1
    assert torch.equal(again["x"], conv["x"])
    mixed = b.Solver(pt, nz, tol=1e-13, mixed=1, max_outer=20).solve(td, x0=tx0)
    assert mixed["info"]["converged"] == 1 and mixed["info"]["true_rel_resid"] <= 1e-13
    assert np.all(oracle.rel_l2_per_stokes(mixed["x"].cpu().numpy(), conv["x"].cpu().numpy()) < 1e-10)
    # two right-hand sides, two start vectors
    X0 = torch.stack([tx0, torch.zeros_like(tx0)]).contiguous()
    two = torch.stack([torch.from_numpy(ds[0]), torch.from_numpy(ds[1])]).to(DEV).contiguous()
    s = b.AsyncSolver(pt, nz, two, x0=X0, fixed_iter=k, tol=0.0)
    for _ in range(10):
        s.step()
        s.stream.synchronize()
        if s.poll()[0]:
            break
    res = s.finish()
    assert np.all(oracle.rel_l2_per_stokes(res["x"][0].cpu().numpy(), x_ref) < 1e-10)
    x_ref1, _ = oracle.pcg(lambda v: oracle.apply_A(opt, noise, v), lambda v: oracle.apply_M(opt, v),
                           oracle.rhs(opt, noise, ds[1]), fixed_iters=k)
    assert np.all(oracle.rel_l2_per_stokes(res["x"][1].cpu().numpy(), x_ref1) < 1e-10)


def test_autotuner_takes_a_cached_choice():
    """A choice put into the tuner's class cache decides the variant of a
    later autotuned solve of that class, and the solve is still right."""
    b = _b()
    w = SMALL_T
    pt, nz, opt, noise, ds = _device_problem(w)
    td = torch.from_numpy(ds[0]).to(DEV)
    ref = b.Solver(pt, nz, tol=1e-10).solve(td)
    cls = {"device": 0, "log2_samples": (w.n_samples).bit_length() - 1, "dtype": b.MM_F64, "arith": b.MM_F64,
           "n_rhs": 1, "ncomp": 3, "lambda": w.lam, "noise_kind": 1}
    for forced in (1, 9):
        b.tune_cache_put([dict(cls, op_variant=forced)])
        nz2 = b.Noise.toeplitz(synth.toeplitz_coeff(w), synth.chunk_offsets(w), DEV)  # no per-handle choice yet
        out = b.Solver(pt, nz2, tol=1e-10, autotune=1).solve(td)
        assert out["info"]["op_variant"] == forced
        assert dict(cls, op_variant=forced) in b.tune_cache_get()
        err = oracle.rel_l2_per_stokes(out["x"].cpu().numpy(), ref["x"].cpu().numpy())
        assert np.all(err < 1e-8), (forced, err)
