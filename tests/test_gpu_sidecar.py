"""GPU parity for the persisted sidecar (the output position of every tile
stored ahead of decoding): fd_sidecar_build against the oracle's sidecar, and
fd_decode_sidecar against the oracle's decode with a sidecar, bit-exact in
status, Arrow offsets and bytes; sidecars that do not match the codes report
FD_ESIDECAR without any write outside the outputs."""
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


def n_codes_of(c):
    return int(c.stats["n_codes"]) if c.codec == "onpair12" else len(c.codes)


class Col:
    """A column on the device with its prepared dictionary."""

    def __init__(self, c):
        import torch
        import paper_2609_15034_amd as fd
        self.c = c
        self.codec = c.codec
        self.n_codes = n_codes_of(c)
        self.n_strings = len(c.code_off) - 1
        codes = c.codes.view(np.int16) if c.codec == "onpair16" else c.codes
        self.codes = torch.from_numpy(np.ascontiguousarray(codes).copy()).cuda()
        self.off = torch.from_numpy(np.ascontiguousarray(c.code_off)).cuda()
        self.d = fd.Dict(c.codec, torch.from_numpy(np.ascontiguousarray(c.dict_bytes, np.uint8)).cuda(),
                         torch.from_numpy(np.ascontiguousarray(c.dict_lens, np.uint8)).cuda())

    def oracle_args(self):
        c = self.c
        return (c.codec, c.codes, c.code_off, c.dict_bytes, c.dict_lens)

    def build(self, tuning=None, async_=False):
        """(status, sidecar tensor, tile_codes) from the GPU."""
        import torch
        import paper_2609_15034_amd as fd
        sb, n = fd.sidecar_layout(self.codec, self.n_codes, self.n_strings, tuning)
        sc = torch.full((n,), -3, dtype=torch.int64, device="cuda")
        ws = fd.alloc_workspace(self.codec, self.n_codes, self.n_strings, tuning)
        status = torch.full((1,), -1, dtype=torch.int32, device="cuda") if async_ else None
        st = fd.sidecar_build_into(self.d, self.codes, self.off, sc, ws, status=status, async_=async_, tuning=tuning,
                                   n_codes=self.n_codes)
        torch.cuda.synchronize()
        if async_:
            assert st == fd.OK
            st = int(status.item())
        return st, sc, sb

    def decode(self, sc, tuning=None, cap=None, async_=False):
        """(status, out_off, out_bytes) from fd_decode_sidecar, guards checked."""
        import torch
        import paper_2609_15034_amd as fd
        if cap is None:
            cap = self.n_codes * (8 if self.codec == "fsst8" else 16)
        g = GuardedOut(cap, self.n_strings + 1, self.off.dtype)
        ws = fd.alloc_workspace(self.codec, self.n_codes, self.n_strings, tuning)
        status = torch.full((1,), -1, dtype=torch.int32, device="cuda") if async_ else None
        st = fd.decode_sidecar_into(self.d, self.codes, self.off, sc, g.off, g.out, ws, status=status, async_=async_,
                                    tuning=tuning, n_codes=self.n_codes)
        torch.cuda.synchronize()
        if async_:
            assert st == fd.OK
            st = int(status.item())
        g.check_guards()
        return st, g.off.cpu().numpy().astype(np.int64), g.out.cpu().numpy()


def check_decode(col, sc, sb, tuning=None, cap=None, async_=False):
    import oracle
    kw = {"n_codes": col.n_codes} if col.codec == "onpair12" else {}
    exp = oracle.decode_with_sidecar(*col.oracle_args(), sc.cpu().numpy(), sb, out_capacity=cap, **kw)
    st, off, out = col.decode(sc, tuning, cap, async_)
    assert st == exp.status, (st, exp.status)
    if exp.status in (0, 4):
        assert np.array_equal(off, exp.out_off)
        assert np.array_equal(out[:len(exp.out_bytes)], exp.out_bytes)
    return exp


@pytest.fixture(scope="module")
def cols(datagen_mod):
    return {"fsst_small": Col(datagen_mod.fsst_small()),
            "fsst_logs": Col(datagen_mod.fsst_logs(target_bytes=8 << 20)),
            "onpair_urls": Col(datagen_mod.onpair_urls(target_bytes=8 << 20, sample_bytes=2 << 20)),
            "onpair12_urls": Col(datagen_mod.onpair12_urls(target_bytes=8 << 20)),
            "fsst12_logs": Col(datagen_mod.fsst12_logs(target_bytes=4 << 20))}


@pytest.mark.parametrize("name", ["fsst_small", "fsst_logs", "onpair_urls", "onpair12_urls", "fsst12_logs"])
@pytest.mark.parametrize("tc", [0, "min", "mid"])
def test_build_and_decode(cols, name, tc):
    """Tile sizes from one 16-byte chunk of codes to the largest."""
    import oracle
    col = cols[name]
    if tc == "min":
        tc = 16 if col.codec == "fsst8" else 8
    elif tc == "mid":
        tc = 1024 if col.codec == "fsst8" else 600
    tu = {"mode": 0, "tile_codes": tc, "grid": 0, "reserved": 0}
    st, sc, sb_used = col.build(tu)
    kw = {"n_codes": col.n_codes} if col.codec == "onpair12" else {}
    est, exp = oracle.sidecar(*col.oracle_args(), sb_used, **kw)
    assert st == est == 0
    assert np.array_equal(sc.cpu().numpy(), exp)
    exp_dec = check_decode(col, sc, sb_used, tu)
    assert exp_dec.status == 0 and np.array_equal(exp_dec.out_bytes, col.c.text)


@pytest.mark.parametrize("grid", [1, 3])
def test_small_grids(cols, grid):
    col = cols["fsst_logs"]
    tu = {"mode": 0, "tile_codes": 0, "grid": grid, "reserved": 0}
    st, sc, sb = col.build(tu)
    assert st == 0
    check_decode(col, sc, sb, tu)


@pytest.mark.parametrize("name", ["fsst_logs", "onpair_urls"])
def test_sidecar_from_source_offsets(cols, name):
    """A sidecar written by an encoder, which knows what each code it emitted
    stands for (a token's length; for FSST-8 an escape stands for nothing and
    its literal for one byte), sampled at every tile start (no decode
    involved), decodes the column."""
    import torch
    import paper_2609_15034_amd as fd
    col = cols[name]
    c = col.c
    T, n = fd.sidecar_layout(col.codec, col.n_codes, col.n_strings)
    lens = c.dict_lens.astype(np.int64)
    if c.codec == "fsst8":
        # escapes and literals: inside a run of 255 the codes alternate escape / literal,
        # starting with an escape at the run's start (every string starts with a code)
        per = np.zeros(len(c.codes), np.int64)
        co = np.asarray(c.code_off, np.int64)
        is_ff = c.codes == 255
        for i in range(c.n_strings):
            a, e = int(co[i]), int(co[i + 1])
            expect_code = True
            for p in range(a, e):
                if expect_code and is_ff[p]:
                    expect_code = False          # an escape: nothing
                elif not expect_code:
                    per[p] = 1                   # its literal
                    expect_code = True
                else:
                    per[p] = lens[c.codes[p]]
    else:
        per = lens[c.codes]
    cum = np.concatenate([[0], np.cumsum(per)])
    pos = [min(k * T, col.n_codes) for k in range(n - 1)] + [col.n_codes]
    sc = torch.from_numpy(cum[pos].copy()).cuda()
    exp = check_decode(col, sc, T)
    assert exp.status == 0


def corrupt(sc, kind):
    v = sc.cpu().numpy().copy()
    n = len(v)
    if kind == "middle+1":
        v[n // 2] += 1
    elif kind == "first":
        v[0] = 5
    elif kind == "shift":
        v += 5
    elif kind == "negative":
        v[n // 3] = -100
    elif kind == "huge":
        v[n // 2] = 1 << 62
    elif kind == "last+1":
        v[-1] += 1
    elif kind == "swap":
        v[1], v[2] = v[2], v[1]
    elif kind == "shift_2^62":          # consistent differences, the last entry at 2^62
        v += (1 << 62) - v[-1]
    elif kind == "shift_2^63":          # consistent differences up to the largest int64
        v += (1 << 63) - 1 - v[-1]
    return v


@pytest.mark.parametrize("kind", ["middle+1", "first", "shift", "negative", "huge", "last+1", "swap", "shift_2^62",
                                  "shift_2^63"])
@pytest.mark.parametrize("name", ["fsst_logs", "onpair_urls"])
def test_wrong_sidecar(cols, name, kind):
    """ESIDECAR, and no byte outside out_bytes[0, exact decoded size)."""
    import torch
    col = cols[name]
    st, sc, sb = col.build()
    assert st == 0
    bad = torch.from_numpy(corrupt(sc, kind)).cuda()
    exp = check_decode(col, bad, sb, cap=len(col.c.text))
    assert exp.status == 10


def test_capacity_and_async(cols):
    col = cols["onpair12_urls"]
    st, sc, sb = col.build(async_=True)
    assert st == 0
    total = len(col.c.text)
    assert check_decode(col, sc, sb, cap=total - 1).status == 4
    assert check_decode(col, sc, sb, cap=total, async_=True).status == 0
    # a wrong sidecar ranks before ECAPACITY
    import torch
    assert check_decode(col, torch.from_numpy(corrupt(sc, "middle+1")).cuda(), sb, cap=10).status == 10


def test_errors_in_the_data(datagen_mod):
    """The build reports the data error; a decode with the column's earlier
    (now stale) sidecar reports the data error, not ESIDECAR."""
    import oracle
    c = datagen_mod.random_onpair(seed=9, n_codes=1 << 16, n_strings=1000, n_tok=1000)
    good = Col(c)
    st, sc, sb = good.build()
    assert st == 0
    codes = c.codes.copy()
    codes[int(c.code_off[len(c.code_off) // 2])] = len(c.dict_lens)      # not a token
    c2 = type(c)(**{**c.__dict__, "codes": codes})
    bad = Col(c2)
    st2, _, _ = bad.build()
    est, _ = oracle.sidecar("onpair16", codes, c.code_off, c.dict_bytes, c.dict_lens, sb)
    assert st2 == est == 2
    assert check_decode(bad, sc, sb).status == 2


def test_empty_and_one_string(datagen_mod):
    import torch
    import paper_2609_15034_amd as fd
    c = datagen_mod.fsst_small(seed=3)
    col = Col(c)
    import oracle
    for n in (0, 1):
        col.off = torch.from_numpy(np.ascontiguousarray(c.code_off[: n + 1])).cuda()
        col.n_strings = n
        st, sc, sb = col.build()
        est, exp = oracle.sidecar("fsst8", c.codes, c.code_off[: n + 1], c.dict_bytes, c.dict_lens, sb)
        assert st == est == 0 and np.array_equal(sc.cpu().numpy(), exp)
        assert exp[-1] == int(c.text_off[n]) and exp[0] == 0
        st, off, out = col.decode(sc)
        assert st == 0 and off.tolist() == [int(x) for x in c.text_off[: n + 1]]


def test_sidecar_of_another_tiling(cols):
    import paper_2609_15034_amd as fd
    col = cols["fsst_small"]
    st, sc, sb = col.build({"mode": 0, "tile_codes": 16, "grid": 0, "reserved": 0})
    assert st == 0
    tu = {"mode": 0, "tile_codes": 32, "grid": 0, "reserved": 0}
    st, _, _ = col.decode(sc, tu)
    assert st == fd.EINVAL
