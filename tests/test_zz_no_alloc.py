"""The no-allocation entry point (fd_decode_noalloc) against fd_decode_ex on
the same columns, bit-exact in status, offsets and bytes: two calls in a row,
the second with a smaller column, so the static scratch must be reset between
calls; then asynchronous calls, tile sizes, an error in the data, and a column
too large for the scratch (rejected on the host)."""
import numpy as np
import pytest

from gpu_util import GuardedOut

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_15034_amd as fd
    fd.lib()
    yield


def run_both(c, tuning=None, codes=None, async_=False):
    """(status, offsets, bytes) of fd_decode_ex and of fd_decode_noalloc."""
    import torch
    import paper_2609_15034_amd as fd
    codes = c.codes if codes is None else codes
    dev = torch.device("cuda")
    ct = torch.from_numpy(codes.view(np.int16) if c.codec == "onpair16" else codes).to(dev)
    off = torch.from_numpy(np.ascontiguousarray(c.code_off)).to(dev)
    d = fd.Dict(c.codec, torch.from_numpy(c.dict_bytes).to(dev), torch.from_numpy(c.dict_lens).to(dev))
    n_codes = fd.codes_in(c.codec, ct) if c.codec != "onpair12" else int(c.stats["n_codes"])
    cap = n_codes * (8 if c.codec == "fsst8" else 16)
    res = []
    for which in ("ex", "noalloc"):
        g = GuardedOut(cap, c.n_strings + 1, off.dtype)
        st_t = torch.full((1,), -1, dtype=torch.int32, device=dev) if async_ else None
        if which == "ex":
            ws = fd.alloc_workspace(c.codec, n_codes, c.n_strings, tuning)
            st = fd.decode_into(d, ct, off, g.off, g.out, ws, status=st_t, async_=async_, tuning=tuning,
                                n_codes=n_codes)
        else:
            st = fd.decode_noalloc_into(d, ct, off, g.off, g.out, status=st_t, async_=async_, tuning=tuning,
                                        n_codes=n_codes)
        torch.cuda.synchronize()
        if async_:
            assert st == fd.OK
            st = int(st_t.item())
        g.check_guards()
        res.append((st, g.off.cpu().numpy(), g.out.cpu().numpy()))
    return res


def assert_same(c, **kw):
    (s1, o1, b1), (s2, o2, b2) = run_both(c, **kw)
    assert s1 == s2, (s1, s2)
    if s1 in (0, 4):
        assert np.array_equal(o1, o2)
        n = int(o1[-1])
        assert np.array_equal(b1[:n], b2[:n])
    return s1


def test_two_calls_second_smaller(datagen_mod):
    """A large column, then a smaller one: the second must not see the first's
    tile totals, look-back states or coarse index in the shared scratch."""
    big = datagen_mod.fsst_logs(target_bytes=16 << 20)
    small = datagen_mod.fsst_small(seed=7, n_strings=3000)
    assert assert_same(big) == 0
    assert assert_same(small) == 0
    for mode in (0, 1):
        tu = {"mode": mode, "tile_codes": 0, "grid": 0, "reserved": 0}
        assert assert_same(big, tuning=tu) == 0
        assert assert_same(small, tuning=tu) == 0


def test_onpair_and_12bit_then_smaller(datagen_mod):
    for c in (datagen_mod.onpair_urls(target_bytes=8 << 20, sample_bytes=2 << 20),
              datagen_mod.onpair12_urls(target_bytes=4 << 20),
              datagen_mod.onpair_urls(seed=9, target_bytes=256 << 10, sample_bytes=256 << 10)):
        assert assert_same(c, async_=True) == 0


def test_small_tiles_and_errors(datagen_mod):
    c = datagen_mod.fsst_small(seed=11, n_strings=2000)
    assert assert_same(c, tuning={"mode": 0, "tile_codes": 16, "grid": 3, "reserved": 0}) == 0
    bad = c.codes.copy()
    i = int(c.code_off[1000])
    bad[i - 1] = 255                                  # string 999 may now end in an escape
    bad[i + 3] = 255
    st = assert_same(c, codes=bad)
    assert st in (0, 3)


def test_too_large_is_rejected(datagen_mod):
    """A column whose tiles do not fit the 4 MiB scratch: FD_EINVAL, nothing enqueued."""
    import torch
    import paper_2609_15034_amd as fd
    c = datagen_mod.fsst_small(seed=12, n_strings=10)
    d = fd.Dict("fsst8", torch.from_numpy(c.dict_bytes).cuda(), torch.from_numpy(c.dict_lens).cuda())
    codes = torch.from_numpy(c.codes).cuda()
    off = torch.from_numpy(np.ascontiguousarray(c.code_off)).cuda()
    out = torch.empty(16, dtype=torch.uint8, device="cuda")
    oo = torch.empty(11, dtype=off.dtype, device="cuda")
    tu = {"mode": 0, "tile_codes": 16, "grid": 0, "reserved": 0}
    # 300,000 tiles of 16 codes need about 4.8 MB of scratch: rejected on the
    # host (before the buffers, which are far smaller than claimed, are touched)
    assert fd.decode_noalloc_into(d, codes, off, oo, out, tuning=tu, n_codes=16 * 300_000) == fd.EINVAL
    # a claim that fits runs: the real column with the same tiles
    assert fd.decode_noalloc_into(d, codes, off, oo, out[:0], tuning=tu) in (fd.OK, fd.ECAPACITY)
