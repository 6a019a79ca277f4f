"""GPU parity for 12-bit packed codes (OnPair-12, and FSST-12 through the same
path): the HIP decoder (through the C ABI) against the CPU oracle, bit-exact
in status, Arrow offsets and bytes, including unaligned packed streams, odd
code counts, every tuning, errors and batches mixing all three codecs."""
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


def decode12(packed, n_codes, code_off, db, dl, *, misalign=0, tuning=None, cap=None, async_=False):
    """Decode a packed stream on the GPU (a fresh dictionary handle)."""
    import torch
    import paper_2609_15034_amd as fd
    raw = np.ascontiguousarray(packed, np.uint8)
    buf = torch.zeros(len(raw) + misalign + 16, dtype=torch.uint8, device="cuda")
    if len(raw):
        buf[misalign:misalign + len(raw)] = torch.from_numpy(raw.copy()).cuda()
    codes = buf[misalign:misalign + len(raw)]
    off = torch.from_numpy(np.ascontiguousarray(code_off)).cuda()
    d = fd.Dict("onpair12", torch.from_numpy(np.ascontiguousarray(db, np.uint8)).cuda(),
                torch.from_numpy(np.ascontiguousarray(dl, np.uint8)).cuda())
    cap = n_codes * 16 if cap is None else cap
    g = GuardedOut(cap, len(code_off), off.dtype)
    ws = fd.alloc_workspace("onpair12", n_codes, len(code_off) - 1, tuning)
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda") if async_ else None
    st = fd.decode_into(d, codes, off, g.off, g.out, ws, status=status, async_=async_, tuning=tuning,
                        n_codes=n_codes)
    torch.cuda.synchronize()
    if async_:
        assert st == fd.OK
        st = int(status.item())
    g.check_guards()
    return st, g.off.cpu().numpy().astype(np.int64), g.out.cpu().numpy()


def assert_parity12(packed, n_codes, code_off, db, dl, **kw):
    import oracle
    exp = oracle.decode("onpair12", packed, code_off, db, dl, n_codes=n_codes, out_capacity=kw.get("cap"))
    st, off, out = decode12(packed, n_codes, code_off, db, dl, **kw)
    assert st == exp.status, (st, exp.status)
    if exp.status in (0, 4):
        assert np.array_equal(off, exp.out_off)
        assert np.array_equal(out[:len(exp.out_bytes)], exp.out_bytes)
    return exp


@pytest.fixture(scope="module")
def cols(datagen_mod):
    return {"onpair12": datagen_mod.onpair12_urls(target_bytes=8 << 20),
            "fsst12": datagen_mod.fsst12_logs(target_bytes=8 << 20)}


@pytest.mark.parametrize("name", ["onpair12", "fsst12"])
def test_columns_8mib(cols, name):
    c = cols[name]
    exp = assert_parity12(c.codes, c.stats["n_codes"], c.code_off, c.dict_bytes, c.dict_lens)
    assert np.array_equal(exp.out_bytes, c.text)


@pytest.mark.parametrize("misalign", [1, 2, 3, 5])
def test_unaligned_streams(cols, misalign):
    c = cols["onpair12"]
    assert_parity12(c.codes, c.stats["n_codes"], c.code_off, c.dict_bytes, c.dict_lens, misalign=misalign)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("tc", [0, 8, 56, 2000])
@pytest.mark.parametrize("grid", [0, 3])
def test_tuning(cols, mode, tc, grid):
    c = cols["fsst12"]
    n = 3001                                    # an odd number of strings, a partial last group of codes
    m = int(c.code_off[n])
    import oracle
    codes16 = oracle.unpack12(c.codes[: (m * 12 + 7) // 8 + 2], m)
    packed = oracle.pack12(codes16)
    assert_parity12(packed, m, c.code_off[: n + 1], c.dict_bytes, c.dict_lens,
                    tuning={"mode": mode, "tile_codes": tc, "grid": grid, "reserved": 0})


@pytest.mark.parametrize("tc", [0, 8, 56, 2000])
@pytest.mark.parametrize("grid", [0, 3])
def test_exact_capacity_three_phases(cols, tc, grid):
    """Mode 1 with the output buffer exactly the decoded size: FSST-12's short
    tokens (under 3.5 bytes per code) take the expand pass with the 16 KiB
    staging window, OnPair-12's the 32 KiB one; one byte less is ECAPACITY."""
    import oracle
    tu = {"mode": 1, "tile_codes": tc, "grid": grid, "reserved": 0}
    for name in ("fsst12", "onpair12"):
        c = cols[name]
        n = 4001
        m = int(c.code_off[n])
        packed = oracle.pack12(oracle.unpack12(c.codes, c.stats["n_codes"])[:m])
        exact = len(oracle.decode("onpair12", packed, c.code_off[: n + 1], c.dict_bytes, c.dict_lens,
                                  n_codes=m).out_bytes)
        assert (exact <= 3.5 * m) == (name == "fsst12")
        assert_parity12(packed, m, c.code_off[: n + 1], c.dict_bytes, c.dict_lens, tuning=tu, cap=exact)
        exp = assert_parity12(packed, m, c.code_off[: n + 1], c.dict_bytes, c.dict_lens, tuning=tu,
                              cap=exact - 1)
        assert exp.status == 4


@pytest.mark.parametrize("n_codes", [0, 1, 2, 3, 7, 8, 9, 4095, 4097])
def test_code_counts(n_codes):
    """Every phase of the last partial group of 8 codes, against a random
    4,096-token dictionary."""
    import oracle
    rng = np.random.default_rng(n_codes)
    lens = rng.integers(1, 17, 4096).astype(np.uint8)
    db = rng.integers(0, 256, int(lens.sum())).astype(np.uint8)
    codes = rng.integers(0, 4096, n_codes)
    cuts = np.sort(rng.integers(0, n_codes + 1, 5))
    code_off = np.concatenate([[0], cuts, [n_codes]]).astype(np.int64)
    assert_parity12(oracle.pack12(codes), n_codes, code_off, db, lens)


def test_codes_past_the_dictionary(cols):
    """A dictionary smaller than the codes used: EBADCODE at the first bad code."""
    c = cols["onpair12"]
    n = 2000
    m = int(c.code_off[n])
    import oracle
    packed = oracle.pack12(oracle.unpack12(c.codes, c.stats["n_codes"])[:m])
    keep = 300
    db, dl = c.dict_bytes[: int(c.dict_lens[:keep].sum())], c.dict_lens[:keep]
    exp = assert_parity12(packed, m, c.code_off[: n + 1], db, dl)
    assert exp.status == 2


def test_async_and_capacity(cols):
    c = cols["onpair12"]
    n = 500
    m = int(c.code_off[n])
    import oracle
    packed = oracle.pack12(oracle.unpack12(c.codes, c.stats["n_codes"])[:m])
    assert_parity12(packed, m, c.code_off[: n + 1], c.dict_bytes, c.dict_lens, async_=True)
    exp = assert_parity12(packed, m, c.code_off[: n + 1], c.dict_bytes, c.dict_lens, cap=1000)
    assert exp.status == 4


def test_dictionary_limit():
    import torch
    import paper_2609_15034_amd as fd
    lens = torch.ones(4097, dtype=torch.uint8, device="cuda")
    with pytest.raises(fd.DecodeError):
        fd.Dict("onpair12", torch.zeros(4097, dtype=torch.uint8, device="cuda"), lens)
    fd.Dict("onpair12", torch.zeros(4096, dtype=torch.uint8, device="cuda"), lens[:4096])


def test_batch_mixed_codecs(datagen_mod, cols):
    """One batch of FSST-8, OnPair-16 and 12-bit columns: every column equals its
    oracle decode."""
    import torch
    import oracle
    import paper_2609_15034_amd as fd
    srcs = [datagen_mod.fsst_small(n_strings=3000), datagen_mod.onpair_urls(target_bytes=1 << 20, sample_bytes=1 << 20),
            cols["onpair12"], cols["fsst12"]]
    tups, exps = [], []
    for c in srcs:
        codes_np = c.codes.view(np.int16) if c.codec == "onpair16" else c.codes
        d = fd.Dict(c.codec, torch.from_numpy(c.dict_bytes).cuda(), torch.from_numpy(c.dict_lens).cuda())
        codes = torch.from_numpy(codes_np.copy()).cuda()
        off = torch.from_numpy(c.code_off).cuda()
        tups.append((d, codes, off, torch.full((c.n_strings + 1,), -7, dtype=off.dtype, device="cuda"),
                     torch.full((c.decoded_bytes + 64,), 0xA5, dtype=torch.uint8, device="cuda")))
        kw = {"n_codes": c.stats["n_codes"]} if c.codec == "onpair12" else {}
        exps.append(oracle.decode(c.codec, c.codes, c.code_off, c.dict_bytes, c.dict_lens, **kw))
    ws = torch.empty(fd.batch_workspace_size(tups, None), dtype=torch.uint8, device="cuda")
    status = torch.full((len(tups) + 1,), -1, dtype=torch.int32, device="cuda")
    for graph in (False, True, True):
        assert fd.batch_decode(tups, ws, status=status, async_=True, graph=graph) == fd.OK
        torch.cuda.synchronize()
        assert status.cpu().tolist() == [0] * (len(tups) + 1)
        for t, e in zip(tups, exps):
            assert np.array_equal(t[3].cpu().numpy().astype(np.int64), e.out_off)
            out = t[4].cpu().numpy()
            assert np.array_equal(out[:len(e.out_bytes)], e.out_bytes)
            assert np.all(out[len(e.out_bytes):] == 0xA5)
