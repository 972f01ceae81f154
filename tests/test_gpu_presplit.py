"""b stored pre-split (rif_presplit_b) for the reduced-precision modes.

The half transform splits b on load with the same arithmetic and the same
pairing of consecutive mu as the pre-split kernel, and b is exactly symmetric,
so a build that reads the pre-split b must equal the one that does not,
bitwise, in every output (FP32, split BF16x3 and x6, split FP16x3; rif_build,
rif_build_direct and a batch).  The piece planes themselves are checked
against their definition: the pieces sum to b within the precision of three
(or two) bf16 pieces, or of the fp16 pair hi + lo 2^-11, and the padding is
zero.
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import host, to_dev

pytestmark = pytest.mark.gpu
MODES = [("fp32", 1), ("bf16x3", 2), ("bf16x6", 3), ("fp16x3", 4)]


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2012_15662_amd as rif
    c = rif.Context()
    yield c
    c.close()


def bf16_to_f32(u16):
    return (u16.astype(np.uint32) << 16).view(np.float32)


@pytest.mark.parametrize("mode,prec", MODES)
@pytest.mark.parametrize("shape", [(37, 101, 3, 2, 11), (130, 259, 7, 3, 12), (4, 1, 1, 1, 13)])
def test_build_with_presplit_b_is_bitwise_equal(ctx, mode, prec, shape):
    inst = synth.make_instance(*shape)
    print("case presplit", mode, shape, flush=True)
    t = to_dev(inst)
    bs = ctx.presplit_b(t["b"], prec)
    a = ctx.build(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], inst.n_pairs, inst.n_cwo, prec=prec)
    b = ctx.build(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], inst.n_pairs, inst.n_cwo, prec=prec, b_split=bs)
    ctx.sync()
    for k in ("b_half", "b_mo", "d", "J", "K", "Jn", "Kn", "energy", "lam", "grad"):
        assert np.array_equal(host(a[k]), host(b[k])), k
    da = ctx.build_direct(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], inst.n_pairs, inst.n_cwo, prec=prec)
    db = ctx.build_direct(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], inst.n_pairs, inst.n_cwo, prec=prec,
                          b_split=bs)
    ctx.sync()
    for k in ("energy", "lam", "grad"):
        assert np.array_equal(host(da[k]), host(db[k])), k


@pytest.mark.parametrize("mode,prec", [("bf16x3", 2), ("bf16x6", 3), ("fp16x3", 4)])
@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_presplit_every_tile_variant(ctx, mode, prec, variant):
    """Each tile shape of the kernels that stage piece planes straight into
    LDS (half transform, J^q), against the same build splitting b on load."""
    inst = synth.make_instance(130, 259, 7, 3, 14 + variant)
    print("case presplit variant", mode, variant, flush=True)
    t = to_dev(inst)
    bs = ctx.presplit_b(t["b"], prec)
    ctx.set_tile_variant(variant)
    try:
        a = ctx.build(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], inst.n_pairs, inst.n_cwo, prec=prec)
        b = ctx.build(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], inst.n_pairs, inst.n_cwo, prec=prec,
                      b_split=bs)
        ctx.sync()
    finally:
        ctx.set_tile_variant(-1)
    for k in ("b_half", "Jn", "Kn", "energy", "lam", "grad"):
        assert np.array_equal(host(a[k]), host(b[k])), k


@pytest.mark.parametrize("mode,prec", [("bf16x6", 3), ("fp16x3", 4)])
def test_presplit_bitwise_at_cyclohexane_size(ctx, mode, prec):
    """The launch shapes the bench times; their ragged last tiles stage
    operand rows past the end, which may reach only discarded outputs."""
    inst = synth.workload("c6h12")
    print("case presplit cyclohexane-like", mode, flush=True)
    t = to_dev(inst)
    bs = ctx.presplit_b(t["b"], prec)
    a = ctx.build(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], inst.n_pairs, inst.n_cwo, prec=prec)
    b = ctx.build(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], inst.n_pairs, inst.n_cwo, prec=prec, b_split=bs)
    ctx.sync()
    for k in ("b_half", "Jn", "Kn", "energy", "lam", "grad"):
        assert np.array_equal(host(a[k]), host(b[k])), k
    del bs, a, b


@pytest.mark.parametrize("mode,prec,npc", [("bf16x3", 2, 2), ("bf16x6", 3, 3)])
def test_piece_planes_sum_to_b(ctx, mode, prec, npc):
    inst = synth.make_instance(37, 20, 2, 1, 5)
    t = to_dev(inst)
    raw = host(ctx.presplit_b(t["b"], prec)).view(np.uint16)
    nb, na, ld = inst.n_bf, inst.n_aux, 64
    planes = raw[:npc * na * nb * ld].reshape(npc, na * nb, ld)
    assert np.all(planes[:, :, nb:] == 0)
    total = sum(bf16_to_f32(planes[s, :, :nb]).astype(np.float64) for s in range(npc))
    ref = inst.b.reshape(na * nb, nb)          # row l*n_bf + nu, column mu (b symmetric)
    err = np.max(np.abs(total - ref)) / np.max(np.abs(ref))
    print(mode, "piece-sum error", err, flush=True)
    assert err < (2.0 ** -23 if npc == 3 else 2.0 ** -15)
    # the leading piece is b rounded to bf16 (round to nearest even)
    hi = bf16_to_f32(planes[0, :, :nb]).astype(np.float64)
    assert np.max(np.abs(hi - ref) / np.maximum(np.abs(ref), 1e-300)) <= 2.0 ** -8 * 1.0001


def test_fp16_planes_sum_to_b(ctx):
    """FP16x3 planes: hi = fp16(b) (round to nearest even, numpy's float16
    conversion of the FP32 value) and lo with hi + lo 2^-11 = b to about 2^-22."""
    import paper_2012_15662_amd as rif
    inst = synth.make_instance(37, 20, 2, 1, 5)
    t = to_dev(inst)
    raw = host(ctx.presplit_b(t["b"], rif.FP16X3)).view(np.uint16)
    nb, na, ld = inst.n_bf, inst.n_aux, 64
    planes = raw[:2 * na * nb * ld].reshape(2, na * nb, ld)
    assert np.all(planes[:, :, nb:] == 0)
    hi = planes[0, :, :nb].view(np.float16).astype(np.float64)
    lo = planes[1, :, :nb].view(np.float16).astype(np.float64)
    ref = inst.b.reshape(na * nb, nb)
    assert np.array_equal(hi, ref.astype(np.float32).astype(np.float16).astype(np.float64))
    err = np.max(np.abs(hi + lo / 2048.0 - ref)) / np.max(np.abs(ref))
    print("fp16x3 piece-sum error", err, flush=True)
    assert err < 2.0 ** -21


def test_fp32_copy_and_errors(ctx):
    import torch
    import paper_2012_15662_amd as rif
    inst = synth.make_instance(20, 30, 2, 1, 6)
    t = to_dev(inst)
    f = host(ctx.presplit_b(t["b"], rif.FP32)).view(np.float32)
    assert np.array_equal(f, inst.b.astype(np.float32).ravel())
    with pytest.raises(rif.RifError):
        ctx.presplit_b(t["b"], rif.FP64)
    assert ctx.lib.rif_presplit_b_bytes(20, 30, rif.FP64) == 0
    # the half-transform region, then the J^q region (n_aux rounded up to 32)
    assert ctx.lib.rif_presplit_b_bytes(20, 30, rif.BF16X6) == 3 * 30 * 20 * 32 * 2 + 3 * 20 * 20 * 32 * 2
    assert ctx.lib.rif_presplit_b_bytes(20, 30, rif.FP16X3) == 2 * 30 * 20 * 32 * 2 + 2 * 20 * 20 * 32 * 2


@pytest.mark.parametrize("prec", [1, 3, 4])
def test_batch_with_presplit_b(ctx, prec):
    insts = [synth.make_instance(60 + 17 * i, 2 * (60 + 17 * i), 3 + i, 2, 70 + i) for i in range(3)]
    items_a, items_b, outs = [], [], []
    for inst in insts:
        t = to_dev(inst)
        t_b = dict(t)
        t_b["b_split"] = ctx.presplit_b(t["b"], prec)
        items_a.append((t, inst.n_pairs, inst.n_cwo, None))
        items_b.append((t_b, inst.n_pairs, inst.n_cwo, None))
    ba = ctx.batch(items_a, prec=prec)
    bb = ctx.batch(items_b, prec=prec)
    ba.run()
    bb.run()
    ctx.sync()
    for oa, ob in zip(ba.outs, bb.outs):
        for k in ("energy", "lam", "grad", "Jn", "Kn"):
            assert np.array_equal(host(oa[k]), host(ob[k])), k


@pytest.mark.parametrize("mode,prec,npc", [("bf16x3", 2, 2), ("bf16x6", 3, 3), ("fp16x3", 4, 2)])
def test_jq_planes_hold_b_by_aux_index(ctx, mode, prec, npc):
    """The second region: plane s, row mu*n_bf + nu, k = l contiguous (n_aux
    rounded up to 32, zero beyond), each element the same pieces as the first
    region's copy of the same b value (one split, two layouts)."""
    inst = synth.make_instance(37, 45, 2, 1, 7)
    t = to_dev(inst)
    raw = host(ctx.presplit_b(t["b"], prec)).view(np.uint16)
    nb, na, ld, lj = inst.n_bf, inst.n_aux, 64, 64
    first = raw[:npc * na * nb * ld].reshape(npc, na, nb, ld)[:, :, :, :nb]     # [s][l][nu][mu]
    second = raw[npc * na * nb * ld:].reshape(npc, nb, nb, lj)                 # [s][mu][nu][l]
    assert raw.size == npc * na * nb * ld + npc * nb * nb * lj
    assert np.all(second[:, :, :, na:] == 0)
    # second[s][mu][nu][l] = piece s of b[l][mu][nu] = first[s][l][nu][mu]
    assert np.array_equal(second[:, :, :, :na], first.transpose(0, 3, 2, 1))
