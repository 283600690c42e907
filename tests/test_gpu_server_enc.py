"""ServerEnc (Alg. 2) on the device, through the C ABI, against the oracle:
bit-exact over every slot at small shapes (out of place with 16-byte and
4-byte alignment, in place), and on sampled records at a full-size shape."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import server_enc as SE
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    from paper_2506_12761_amd import vlp
    ctx = vlp.Context(0)
    yield vlp, ctx
    ctx.close()


def _inputs(mode, M, l, lS, d, seed):
    g = synth.stream(seed, "se-gpu:%s" % mode)
    if mode == "intv":
        loc = synth.signed_ints(g, (M, d, 2), l)
    elif mode == "cov":
        loc = synth.signed_ints(g, (M, d), l)
    else:
        loc = synth.unsigned_ints(g, (M,), l).astype(np.uint64)
    pay = (synth.uniform_u32(g, (M, lS)) % 256).astype(np.uint8)
    pay[:, ::3] = 0
    pk_loc = synth.uniform_ciphertexts(seed, "pk_loc", SE.loc_slots(mode, M, l, d))
    pk_pay = synth.uniform_ciphertexts(seed, "pk_pay", (M, lS))
    return loc, pay, pk_loc, pk_pay


def _offset_copy(ctx, arr, words_offset):
    """Device copy of a uint32 array starting `words_offset` words into a larger buffer."""
    flat = np.zeros(arr.size + words_offset, np.uint32)
    flat[words_offset:] = arr.reshape(-1)
    t = ctx.tensor(flat)
    return t, t[words_offset:].view(arr.shape)


@pytest.mark.parametrize("mode,M,l,lS,d", [("intv", 3, 5, 4, 2), ("cov", 5, 7, 3, 1), ("cov", 4, 64, 2, 2),
                                           ("idm", 7, 9, 0, 1), ("idm", 1, 1, 1, 1), ("idm", 6, 64, 5, 1)])
@pytest.mark.parametrize("where", ["copy", "inplace", "unaligned"])
def test_server_enc_parity(gpu, mode, M, l, lS, d, where):
    vlp, ctx = gpu
    loc, pay, pk_loc, pk_pay = _inputs(mode, M, l, lS, d, seed=M * 131 + l)
    want_loc = SE.server_enc_loc(mode, l, pk_loc, loc)
    want_pay = SE.server_enc_pay(pk_pay, pay)
    sh = vlp.make_shape(mode, M, l, lS, d)
    d_loc, d_pay = ctx.array(loc), (ctx.array(pay) if lS else None)
    if where == "unaligned":
        keep1, d_pk_loc = _offset_copy(ctx, pk_loc, 1)
        keep2, d_pk_pay = _offset_copy(ctx, pk_pay, 3)
        keep3, o_loc = _offset_copy(ctx, np.zeros_like(pk_loc), 2)
        keep4, o_pay = _offset_copy(ctx, np.zeros_like(pk_pay), 1)
    else:
        d_pk_loc, d_pk_pay = ctx.tensor(pk_loc), ctx.tensor(pk_pay)
        if where == "inplace":
            o_loc, o_pay = d_pk_loc, d_pk_pay
        else:
            o_loc, o_pay = ctx.empty(*pk_loc.shape), ctx.empty(*pk_pay.shape)
    vlp.vlp_server_encrypt(ctx.ctx, sh, d_pk_loc, d_pk_pay if lS else None, d_loc, d_pay,
                           o_loc, o_pay if lS else None)
    ctx.sync()
    assert np.array_equal(ctx.to_host(o_loc), want_loc)
    if lS:
        assert np.array_equal(ctx.to_host(o_pay), want_pay)


def test_server_enc_rejects_bad_arguments(gpu):
    vlp, ctx = gpu
    loc, pay, pk_loc, pk_pay = _inputs("idm", 4, 8, 2, 1, seed=9)
    sh = vlp.make_shape("idm", 4, 8, 2, 1)
    d_pk_loc, d_pk_pay = ctx.tensor(pk_loc), ctx.tensor(pk_pay)
    d_loc, d_pay = ctx.array(loc), ctx.array(pay)
    o_loc = ctx.empty(*pk_loc.shape)
    with pytest.raises(vlp.VlpError) as e:  # payload arrays missing while l_S > 0
        vlp.vlp_server_encrypt(ctx.ctx, sh, d_pk_loc, None, d_loc, None, o_loc, None)
    assert e.value.status == vlp.VLP_EINVAL
    with pytest.raises(vlp.VlpError) as e:  # output shifted one record into its public key
        vlp.vlp_server_encrypt(ctx.ctx, sh, d_pk_loc, d_pk_pay, d_loc, d_pay, d_pk_loc[1:], ctx.empty(*pk_pay.shape))
    assert e.value.status == vlp.VLP_EINVAL
    with pytest.raises(vlp.VlpError) as e:  # l_I out of range
        vlp.vlp_server_encrypt(ctx.ctx, vlp.make_shape("idm", 4, 65, 2, 1), d_pk_loc, d_pk_pay, d_loc, d_pay, o_loc,
                               ctx.empty(*pk_pay.shape))
    assert e.value.status == vlp.VLP_EINVAL


def test_server_enc_full_size_sampled(gpu):
    """4,096 records of 32-bit identifiers with 16 payload bits (196,608
    ciphertexts, 0.5 GB of public key: every workgroup of the grid-stride
    copy loops many times), out of place; 24 sampled records checked against
    the oracle, and every body word checked against Ecd of its bit."""
    vlp, ctx = gpu
    mode, M, l, lS, d = "idm", 4096, 32, 16, 1
    loc, pay, pk_loc, pk_pay = _inputs(mode, M, l, lS, d, seed=77)
    sh = vlp.make_shape(mode, M, l, lS, d)
    d_pk_loc, d_pk_pay = ctx.tensor(pk_loc), ctx.tensor(pk_pay)
    o_loc, o_pay = ctx.empty(*pk_loc.shape), ctx.empty(*pk_pay.shape)
    vlp.vlp_server_encrypt(ctx.ctx, sh, d_pk_loc, d_pk_pay, ctx.array(loc), ctx.array(pay), o_loc, o_pay)
    ctx.sync()
    got_loc, got_pay = ctx.to_host(o_loc), ctx.to_host(o_pay)
    idx = np.sort(synth.stream(78, "sample").choice(M, 24, replace=False))
    idx[-1] = M - 1
    assert np.array_equal(got_loc[idx], SE.server_enc_loc(mode, l, pk_loc[idx], loc[idx]))
    assert np.array_equal(got_pay[idx], SE.server_enc_pay(pk_pay[idx], pay[idx]))
    # Masks are copied; body - pk body is Ecd of the slot's bit (any size).
    assert np.array_equal(got_loc[..., :O.n], pk_loc[..., :O.n])
    bits = (loc[:, None].astype(np.uint64) >> np.arange(l, dtype=np.uint64)[None, :]) & np.uint64(1)
    diff = (got_loc[..., O.n].astype(np.int64) - pk_loc[..., O.n].astype(np.int64)) % 2**32
    assert np.array_equal(diff, np.where(bits == 1, O.MU, 2**32 - O.MU))
    diff = (got_pay[..., O.n].astype(np.int64) - pk_pay[..., O.n].astype(np.int64)) % 2**32
    assert np.array_equal(diff, np.where(pay != 0, O.MU, 2**32 - O.MU))
