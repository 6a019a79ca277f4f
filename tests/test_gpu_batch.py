"""GPU parity of batch_decode: many columns of mixed codecs and offset widths in
one submission (and as a replayed HIP graph) against the CPU oracle, column by
column, bit-exact in status, Arrow offsets and bytes."""
import numpy as np
import pytest

from gpu_util import CANARY, GUARD

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_15034_amd as fd
    fd.lib()
    yield


class Col:
    """A column on the device with guarded outputs, plus its oracle result."""

    def __init__(self, codec, codes, code_off, dict_bytes, dict_lens, d=None, cap=None, idx=np.int64):
        import torch
        import oracle
        import paper_2609_15034_amd as fd
        self.codec = codec
        self.code_off_np = np.ascontiguousarray(code_off, idx)
        self.codes_np = np.ascontiguousarray(codes)
        maxlen = 8 if codec == "fsst8" else 16
        self.cap = len(codes) * maxlen if cap is None else cap
        self.exp = oracle.decode(codec, self.codes_np, self.code_off_np, dict_bytes, dict_lens,
                                 out_capacity=self.cap)
        self.codes = torch.from_numpy(self.codes_np.copy()).cuda()
        if codec == "onpair16":
            self.codes = self.codes.view(torch.int16)
        self.code_off = torch.from_numpy(self.code_off_np.copy()).cuda()
        if d is None:
            db = torch.from_numpy(np.ascontiguousarray(dict_bytes, np.uint8) if len(dict_bytes)
                                  else np.zeros(1, np.uint8)).cuda()
            d = fd.Dict(codec, db, torch.from_numpy(np.ascontiguousarray(dict_lens, np.uint8)).cuda())
        self.d = d
        n = len(self.code_off_np)
        self.buf = torch.full((GUARD + self.cap + GUARD,), CANARY, dtype=torch.uint8, device="cuda")
        self.out = self.buf[GUARD:GUARD + self.cap]
        self.obuf = torch.full((n + 32,), -7, dtype=self.code_off.dtype, device="cuda")
        self.off = self.obuf[16:16 + n]

    def tup(self):
        return (self.d, self.codes, self.code_off, self.off, self.out if self.cap else None)

    def clear(self):
        self.buf.fill_(CANARY)
        self.obuf.fill_(-7)

    def check(self, st):
        assert st == self.exp.status, (self.codec, st, self.exp.status)
        b = self.buf.cpu().numpy()
        assert np.all(b[:GUARD] == CANARY) and np.all(b[GUARD + self.cap:] == CANARY), "write outside out_bytes"
        o = self.obuf.cpu().numpy()
        assert np.all(o[:16] == -7) and np.all(o[-16:] == -7), "write outside out_offsets"
        if self.exp.status in (0, 4):
            assert np.array_equal(self.off.cpu().numpy().astype(np.int64), self.exp.out_off)
            n = len(self.exp.out_bytes)
            assert np.array_equal(b[GUARD:GUARD + n], self.exp.out_bytes)


def mixed_columns(datagen_mod):
    """Columns of both codecs and offset widths, from empty to ~1 MiB, sharing
    some dictionaries, one a slice (code_offsets[0] > 0)."""
    cols = []
    s = datagen_mod.fsst_small(seed=41, n_strings=3000)
    cols.append(Col("fsst8", s.codes, s.code_off, s.dict_bytes, s.dict_lens, idx=np.int32))
    cols.append(Col("fsst8", s.codes, s.code_off.astype(np.int64), s.dict_bytes, s.dict_lens, d=cols[0].d))
    lg = datagen_mod.fsst_logs(seed=42, target_bytes=1 << 20, sample_bytes=256 << 10)
    cols.append(Col("fsst8", lg.codes, lg.code_off, lg.dict_bytes, lg.dict_lens))
    # a slice of the log column
    cols.append(Col("fsst8", lg.codes, lg.code_off[100:2101], lg.dict_bytes, lg.dict_lens, d=cols[2].d))
    ur = datagen_mod.onpair_urls(seed=43, target_bytes=1 << 20, sample_bytes=512 << 10)
    cols.append(Col("onpair16", ur.codes, ur.code_off, ur.dict_bytes, ur.dict_lens))
    cols.append(Col("onpair16", ur.codes, ur.code_off.astype(np.int32), ur.dict_bytes, ur.dict_lens, d=cols[4].d))
    rnd = datagen_mod.random_onpair(seed=44, n_codes=1 << 15, n_strings=500)
    cols.append(Col("onpair16", rnd.codes, rnd.code_off, rnd.dict_bytes, rnd.dict_lens))
    # degenerate: no strings, empty strings only, one code
    cols.append(Col("fsst8", np.zeros(0, np.uint8), np.zeros(1, np.int64), s.dict_bytes, s.dict_lens, d=cols[0].d))
    cols.append(Col("onpair16", np.zeros(0, np.uint16), np.zeros(5, np.int32), ur.dict_bytes, ur.dict_lens,
                    d=cols[4].d))
    cols.append(Col("fsst8", np.array([3], np.uint8), np.array([0, 1], np.int32), s.dict_bytes, s.dict_lens,
                    d=cols[0].d))
    return cols


def run_batch(cols, tuning=None, graph=False, async_=True):
    import torch
    import paper_2609_15034_amd as fd
    tups = [c.tup() for c in cols]
    ws = torch.empty(fd.batch_workspace_size(tups, tuning), dtype=torch.uint8, device="cuda")
    status = torch.full((len(cols) + 1,), -1, dtype=torch.int32, device="cuda")
    rc = fd.batch_decode(tups, ws, status=status, tuning=tuning, graph=graph, async_=async_)
    torch.cuda.synchronize()
    return rc, status.cpu().numpy(), ws, status


@pytest.mark.parametrize("tuning", [None, {"mode": 0, "tile_codes": 0, "grid": 0, "reserved": 0},
                                    {"mode": 0, "tile_codes": 48, "grid": 5, "reserved": 0},
                                    {"mode": 1, "tile_codes": 0, "grid": 0, "reserved": 0},
                                    {"mode": 1, "tile_codes": 48, "grid": 5, "reserved": 0},
                                    {"mode": 1, "tile_codes": 16, "grid": 0, "reserved": 0}])
def test_batch_matches_oracle(datagen_mod, tuning):
    cols = mixed_columns(datagen_mod)
    rc, st, _, _ = run_batch(cols, tuning=tuning)
    assert rc == 0
    for c, s in zip(cols, st[:-1]):
        c.check(int(s))
    assert st[-1] == 0


def test_batch_sync_return(datagen_mod):
    cols = mixed_columns(datagen_mod)[:4]
    rc, st, _, _ = run_batch(cols, async_=False)
    assert rc == 0 and np.all(st == 0)
    for c in cols:
        c.check(0)


@pytest.mark.parametrize("mode", [0, 1])
def test_batch_errors_per_column(datagen_mod, mode):
    """Each column reports its own status; the overall status is the first
    error in column order; a column's error does not touch the others."""
    s = datagen_mod.fsst_small(seed=45, n_strings=800)
    good = Col("fsst8", s.codes, s.code_off, s.dict_bytes, s.dict_lens)
    bad_codes = s.codes.copy()
    bad_codes[len(bad_codes) // 2] = 254           # not a symbol of a 253-symbol table
    db, dl = s.dict_bytes, s.dict_lens
    keep = int(dl[:253].sum())
    bad = Col("fsst8", bad_codes, s.code_off, db[:keep], dl[:253])
    small = Col("fsst8", s.codes, s.code_off, s.dict_bytes, s.dict_lens, d=good.d, cap=100)
    ur = datagen_mod.onpair_urls(seed=46, target_bytes=128 << 10, sample_bytes=128 << 10)
    good2 = Col("onpair16", ur.codes, ur.code_off, ur.dict_bytes, ur.dict_lens)
    cols = [good, small, bad, good2]
    rc, st, _, _ = run_batch(cols, async_=False, tuning={"mode": mode, "tile_codes": 0, "grid": 0, "reserved": 0})
    assert [c.exp.status for c in cols] == [0, 4, 2, 0]
    for c, x in zip(cols, st[:-1]):
        c.check(int(x))
    assert st[-1] == 4 and rc == 4


@pytest.mark.parametrize("mode", [None, 0, 1])
def test_batch_graph_replays(datagen_mod, mode):
    """FD_GRAPH: the first call records a graph, later calls replay it; every
    replay (with other device work in between) gives the oracle's result."""
    import torch
    import paper_2609_15034_amd as fd
    cols = mixed_columns(datagen_mod)
    tups = [c.tup() for c in cols]
    tu = None if mode is None else {"mode": mode, "tile_codes": 0, "grid": 0, "reserved": 0}
    ws = torch.empty(fd.batch_workspace_size(tups, tu), dtype=torch.uint8, device="cuda")
    status = torch.full((len(cols) + 1,), -1, dtype=torch.int32, device="cuda")
    noise = torch.randn(1 << 20, device="cuda")
    for rep in range(4):
        for c in cols:
            c.clear()
        status.fill_(-1)
        noise.mul_(1.0001).add_(0.5)                   # eager work between replays
        rc = fd.batch_decode(tups, ws, status=status, graph=True, async_=(rep % 2 == 0), tuning=tu)
        torch.cuda.synchronize()
        assert rc == 0
        st = status.cpu().numpy()
        for c, x in zip(cols, st[:-1]):
            c.check(int(x))
        assert st[-1] == 0


def test_batch_equals_single(datagen_mod):
    """A column decoded in a batch is byte-identical to the same column decoded alone."""
    import torch
    import paper_2609_15034_amd as fd
    cols = mixed_columns(datagen_mod)
    run_batch(cols)
    for c in cols[:7]:
        ws = fd.alloc_workspace(c.codec, c.codes.numel(), c.code_off.numel() - 1)
        out = torch.empty_like(c.out)
        off = torch.empty_like(c.off)
        assert fd.decode_into(c.d, c.codes, c.code_off, off, out, ws) == 0
        assert torch.equal(off, c.off)
        n = int(c.exp.out_off[-1])
        assert torch.equal(out[:n], c.out[:n])


@pytest.mark.parametrize("mode", [None, 1])
def test_batch_many_small_columns(datagen_mod, mode):
    """256 columns, sizes log-uniform over two decades, codecs alternating."""
    rng = np.random.default_rng(47)
    s = datagen_mod.fsst_small(seed=48, n_strings=4000)
    ur = datagen_mod.onpair_urls(seed=49, target_bytes=256 << 10, sample_bytes=256 << 10)
    cols = []
    df = dp = None
    for i in range(256):
        src = s if i % 2 == 0 else ur
        codec = "fsst8" if i % 2 == 0 else "onpair16"
        n = int(np.exp(rng.uniform(np.log(2), np.log(len(src.code_off) - 1))))
        a = int(rng.integers(0, len(src.code_off) - 1 - n + 1))
        off = src.code_off[a:a + n + 1]
        c = Col(codec, src.codes, off.astype(np.int32 if i % 3 == 0 else np.int64), src.dict_bytes, src.dict_lens,
                d=(df if codec == "fsst8" else dp))
        if codec == "fsst8":
            df = c.d
        else:
            dp = c.d
        cols.append(c)
    tu = None if mode is None else {"mode": mode, "tile_codes": 0, "grid": 0, "reserved": 0}
    rc, st, _, _ = run_batch(cols, tuning=tu)
    assert rc == 0
    for c, x in zip(cols, st[:-1]):
        c.check(int(x))


# --------------------------------------------------------------------------- #
# the graph cache: full keys, dictionaries by identity
# --------------------------------------------------------------------------- #
def test_graph_cache_colliding_hashes(datagen_mod):
    """With the cache's hash cut to 0 bits every batch collides: replays of two
    different batches (other columns, other dictionaries, each with its own
    workspace and status) must still each run their own graph, told apart by
    the full key."""
    import torch
    import paper_2609_15034_amd as fd
    a = [Col("fsst8", *cols_of(datagen_mod.fsst_small(seed=71, n_strings=800)))]
    b = [Col("onpair16", *cols_of(datagen_mod.onpair_urls(seed=72, target_bytes=128 << 10,
                                                          sample_bytes=128 << 10)))]
    tu = {"mode": 1, "tile_codes": 0, "grid": 0, "reserved": 0}
    runs = []
    for cols in (a, b):
        tups = [c.tup() for c in cols]
        ws = torch.empty(fd.batch_workspace_size(tups, tu), dtype=torch.uint8, device="cuda")
        status = torch.full((len(cols) + 1,), -1, dtype=torch.int32, device="cuda")
        runs.append((cols, tups, ws, status))
    fd.debug_graph_hash_bits(0)
    try:
        for rep in range(3):                        # recorded on the first pass, replayed after
            for cols, tups, ws, status in runs:
                for c in cols:
                    c.clear()
                status.fill_(-1)
                assert fd.batch_decode(tups, ws, status=status, tuning=tu, graph=True, async_=True) == fd.OK
                torch.cuda.synchronize()
                st = status.cpu().numpy()
                for c, s_ in zip(cols, st[:-1]):
                    c.check(int(s_))
        assert fd.debug_graph_count() >= 2
    finally:
        fd.debug_graph_hash_bits(64)


def test_graph_cache_forgets_destroyed_dictionaries(datagen_mod):
    """A graph recorded for a dictionary is dropped when the dictionary is
    destroyed; a new dictionary (possibly at the recycled address, with other
    symbols) decodes its own column correctly through the same buffers."""
    import gc
    import torch
    import paper_2609_15034_amd as fd
    c1 = datagen_mod.fsst_small(seed=81, n_strings=600)
    c2 = datagen_mod.fsst_small(seed=82, n_strings=600)    # another table, other codes
    col = Col("fsst8", *cols_of(c1))
    tu = {"mode": 0, "tile_codes": 0, "grid": 0, "reserved": 0}
    rc, st, _, _ = run_batch([col], tuning=tu, graph=True)
    col.check(int(st[0]))
    n_before = fd.debug_graph_count()
    del col.d
    gc.collect()
    assert fd.debug_graph_count() < n_before                # the graph that read it is gone
    # the second column in new buffers, with a dictionary created afterwards
    col2 = Col("fsst8", *cols_of(c2))
    for _ in range(2):
        col2.clear()
        rc, st, _, _ = run_batch([col2], tuning=tu, graph=True)
        col2.check(int(st[0]))
    torch.cuda.synchronize()


def cols_of(c):
    return c.codes, c.code_off, c.dict_bytes, c.dict_lens
