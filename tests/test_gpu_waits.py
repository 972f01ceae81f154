"""Failure handling of the one-launch kernels, forced from the host.

The tridiagonal reduction of rif_orbital_step and the factorisation of
rif_prepare_b exchange values between workgroups through slots that each
consumer polls, each wait bounded.  rif_set_wait_limit(-1) makes every such
wait give up at once: every workgroup returns, the kernels end normally, and
the call reports it -- info = -1 from rif_orbital_step, an error (status 2)
from rif_pnof_optimize, b all NaN from rif_prepare_b.  After the default limit
is restored the same calls give the results of a run that never failed.
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import host, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2012_15662_amd as rif
    c = rif.Context()
    yield c
    c.set_wait_limit()
    c.set_eigensolver(rif.EIG_AUTO)
    c.close()


@pytest.mark.parametrize("kind", [2, 3])   # the reduction, then dstedc or the library's divide and conquer
def test_orbital_step_reports_a_timed_out_reduction(ctx, kind):
    import torch
    print("case waits: orbital step, eigensolver", kind, flush=True)
    inst = synth.make_instance(37, 101, 3, 2, 11)
    t = to_dev(inst)
    out = ctx.build(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], inst.n_pairs, inst.n_cwo)
    W = inst.occ.size
    ctx.set_eigensolver(kind)
    info = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    C_ref = t["C"].clone()
    w_ref = ctx.orbital_step(out["lam"], C_ref, W, info=info)
    ctx.sync()
    assert int(host(info)[0]) == 0
    ctx.set_wait_limit(-1)
    C_bad = t["C"].clone()
    ctx.orbital_step(out["lam"], C_bad, W, info=info)
    ctx.sync()
    assert int(host(info)[0]) == -1
    ctx.set_wait_limit()
    C = t["C"].clone()
    w = ctx.orbital_step(out["lam"], C, W, info=info)
    ctx.sync()
    assert int(host(info)[0]) == 0
    assert np.array_equal(host(w), host(w_ref))
    assert np.array_equal(host(C), host(C_ref))


@pytest.mark.parametrize("kind", [2, 3])
def test_optimisation_loop_fails_on_a_timed_out_reduction(ctx, kind):
    import torch
    import paper_2012_15662_amd as rif
    print("case waits: optimisation loop, eigensolver", kind, flush=True)
    inst = synth.make_instance(20, 40, 2, 1, 41)
    t = to_dev(inst)
    occ = t["occ"].clone()
    gamma = torch.zeros(inst.n_pairs * inst.n_cwo, dtype=torch.float64, device="cuda")
    ctx.set_eigensolver(kind)
    ctx.set_wait_limit(-1)
    try:
        with pytest.raises(rif.RifError) as e:
            ctx.optimize(t["b"], t["C"].clone(), t["H"], occ, gamma, t["pair_of"], inst.n_pairs, inst.n_cwo,
                         max_outer=1, max_inner=3)
        assert e.value.status == -3   # RIF_EHIP
    finally:
        ctx.set_wait_limit()
    res, _, _ = ctx.optimize(t["b"], t["C"].clone(), t["H"], t["occ"].clone(), gamma.zero_(), t["pair_of"],
                             inst.n_pairs, inst.n_cwo, max_outer=1, max_inner=3)
    assert res["inner_total"] == 3 and np.isfinite(res["energy"])


def test_prepare_b_poisons_b_on_a_timed_out_factorisation(ctx):
    import torch
    print("case waits: b preparation", flush=True)
    n_bf, n_aux = 9, 60
    G = torch.from_numpy(synth.make_metric(n_aux, 5, cond=1e4)).cuda()
    T = torch.from_numpy(synth.make_three_centre(n_bf, n_aux, 6)).cuda()
    b_ref = host(ctx.prepare_b(T, G))
    ctx.set_wait_limit(-1)
    try:
        b_bad = host(ctx.prepare_b(T, G))
    finally:
        ctx.set_wait_limit()
    assert np.all(np.isnan(b_bad))
    b = host(ctx.prepare_b(T, G))
    assert np.all(np.isfinite(b_ref)) and np.array_equal(b, b_ref)
