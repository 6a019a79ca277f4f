"""GPU parity: the HIP decoder (through the C ABI) against the CPU oracle,
bit-exact in status, Arrow offsets and bytes, on seeded inputs."""
import numpy as np
import pytest

from gpu_util import assert_parity, gpu_decode

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_15034_amd as fd
    fd.lib()   # raises when the library is not built
    yield


def pack(tokens):
    lens = np.array([len(t) for t in tokens], np.uint8)
    return np.frombuffer(b"".join(tokens), np.uint8).copy(), lens


# --------------------------------------------------------------------------- #
# workload recipes at test sizes
# --------------------------------------------------------------------------- #
@pytest.mark.parametrize("via", ["dict", "oneshot"])
def test_fsst_small(datagen_mod, via):
    c = datagen_mod.fsst_small()
    assert_parity("fsst8", c.codes, c.code_off, c.dict_bytes, c.dict_lens, via=via)


@pytest.mark.parametrize("via", ["dict", "oneshot"])
def test_fsst_logs_8mib(datagen_mod, via):
    c = datagen_mod.fsst_logs(target_bytes=8 << 20)
    exp = assert_parity("fsst8", c.codes, c.code_off, c.dict_bytes, c.dict_lens, via=via)
    assert np.array_equal(exp.out_bytes, c.text)


@pytest.mark.parametrize("via", ["dict", "oneshot"])
def test_onpair_urls_8mib(datagen_mod, via):
    c = datagen_mod.onpair_urls(target_bytes=8 << 20, sample_bytes=2 << 20)
    exp = assert_parity("onpair16", c.codes, c.code_off, c.dict_bytes, c.dict_lens, via=via)
    assert np.array_equal(exp.out_bytes, c.text)


@pytest.mark.parametrize("tuning", [None, {"mode": 1, "tile_codes": 0, "grid": 0, "reserved": 0},
                                    {"mode": 1, "tile_codes": 64, "grid": 5, "reserved": 0}])
def test_random_full_dictionary(datagen_mod, tuning):
    """All 65,536 tokens, lengths 1-16 uniform, codes uniform: in three phases
    the totals take every length from the nibble table's dword reads."""
    c = datagen_mod.random_onpair(n_codes=1 << 20, n_strings=20_000)
    assert len(c.dict_lens) == 65536 and set(np.unique(c.dict_lens)) == set(range(1, 17))
    assert_parity("onpair16", c.codes, c.code_off, c.dict_bytes, c.dict_lens, tuning=tuning)


# --------------------------------------------------------------------------- #
# tuning: modes, tiny tiles (strings across many tiles, long look-back
# chains), small grids
# --------------------------------------------------------------------------- #
def tu(mode=0, tc=0, grid=0):
    return {"mode": mode, "tile_codes": tc, "grid": grid, "reserved": 0}


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("tc", [0, 16, 48, 272, 2048])
@pytest.mark.parametrize("grid", [0, 1, 7])
def test_tuning_fsst(datagen_mod, mode, tc, grid):
    c = datagen_mod.fsst_small(seed=4, n_strings=3000)
    assert_parity("fsst8", c.codes, c.code_off, c.dict_bytes, c.dict_lens, tuning=tu(mode, tc, grid))


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("tc", [0, 8, 40, 1000])
@pytest.mark.parametrize("grid", [0, 2])
def test_tuning_onpair(datagen_mod, mode, tc, grid):
    c = datagen_mod.onpair_urls(seed=5, target_bytes=1 << 20, sample_bytes=1 << 20)
    assert_parity("onpair16", c.codes, c.code_off, c.dict_bytes, c.dict_lens, tuning=tu(mode, tc, grid))


# --------------------------------------------------------------------------- #
# FSST-8 escapes: runs of 255 of every length across lane / wave / tile edges
# --------------------------------------------------------------------------- #
def _ff_column(seed, n_strings, max_run=300):
    """Strings whose codes contain runs of 255 of every length 0..max_run.  A
    run of even length 2m decodes to m bytes 0xFF; a run of odd length is
    followed by one more byte that becomes a literal."""
    rng = np.random.default_rng(seed)
    strings = []
    run = 0
    while len(strings) < n_strings:
        parts = bytearray()
        for _ in range(int(rng.integers(0, 4))):
            parts += bytes(rng.integers(0, 3, size=int(rng.integers(0, 20))).astype(np.uint8))  # codes 0..2
            L = run % (max_run + 1)
            run += 1
            parts += b"\xff" * L
            if L % 2 == 1:
                parts.append(int(rng.choice([0, 1, 0xFF, 0x41, 200])))   # the literal
        strings.append(bytes(parts))
    codes = np.frombuffer(b"".join(strings), np.uint8).copy()
    off = np.concatenate([[0], np.cumsum([len(s) for s in strings])]).astype(np.int64)
    return codes, off


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("tc", [0, 16, 32, 112])
def test_ff_runs(tc, mode):
    """Runs of 255 of every length up to 300, across lane, wave and (with
    small tiles) tile starts: a tile that starts inside a run takes its parity
    from the bytes before it."""
    codes, off = _ff_column(7, 2500)
    db, dl = pack([b"x", b"yz", b"0123456"])
    assert_parity("fsst8", codes, off, db, dl, tuning=tu(mode, tc))


@pytest.mark.parametrize("mode", [0, 1])
def test_ff_run_longer_than_a_pass(mode):
    """One string whose code stream is a 255 run longer than one pass (8192
    codes) and than the three-phase totals' per-wave step (2048 codes),
    followed by a literal: parity carried across passes, lanes and steps."""
    for L in (2047, 2048, 2049, 4095, 4096, 4097, 9001, 20000):
        codes = np.frombuffer(b"\x00" + b"\xff" * L + (b"\x01" if L % 2 else b"") + b"\x02", np.uint8).copy()
        off = np.array([0, len(codes)], np.int64)
        db, dl = pack([b"a", b"bc", b"def"])
        assert_parity("fsst8", codes, off, db, dl, tuning=tu(mode))
        assert_parity("fsst8", codes, off, db, dl, tuning=tu(mode, 16))


def _edge_escape_column(seed, n_tiles=5, T=8176):
    """Isolated escapes on the last code of lanes (32 codes), of the totals'
    per-wave steps (2048 codes) and of tiles, so that the literal is the
    first code of the next lane, step or tile; in some steps also a literal
    255 (255 255), and in one a literal 255 carried into a step from the
    escape that ends the step before.  Strings never end between an escape
    and its literal."""
    rng = np.random.default_rng(seed)
    n = n_tiles * T + 37
    codes = rng.integers(0, 3, size=n).astype(np.uint8)
    esc = set()
    for t in range(n_tiles):
        base = t * T
        for p in range(base + 31, min(base + T, n - 1), 32 * int(rng.integers(1, 5))):
            esc.add(p)                                   # lane edges
        for r in range(1, 5):
            if base + 2048 * r - 1 < n - 1:
                esc.add(base + 2048 * r - 1)             # step edges
        if base + T - 1 < n - 1:
            esc.add(base + T - 1)                        # tile edges
    for p in sorted(esc):
        codes[p] = 255
        codes[p + 1] = int(rng.choice([0, 1, 0x41, 200]))
    # literal 255s: an escape pair inside step 1 of tile 1, and the literal of
    # the escape ending step 0 of tile 3 (carried into step 1)
    for p in (T + 2048 + 100, 3 * T + 2047):
        codes[p] = 255
        codes[p + 1] = 255
        esc.add(p)
    lit = {p + 1 for p in esc}
    cuts = [0]
    pos = 0
    while True:
        pos += int(rng.integers(1, 90))
        if pos >= n:
            break
        if pos not in lit:
            cuts.append(pos)
    cuts.append(n)
    return codes, np.array(cuts, np.int64)


@pytest.mark.parametrize("mis", [0, 5])
@pytest.mark.parametrize("mode", [0, 1])
def test_escapes_on_lane_step_and_tile_edges(mode, mis):
    """Escapes whose literals open the next lane, totals step or tile, with
    and without a literal 255 in the same step (mode 1's totals take a
    shortcut where no two 255 codes are adjacent)."""
    codes, off = _edge_escape_column(41)
    db, dl = pack([b"a", b"bc", b"defgh"])
    assert_parity("fsst8", codes, off, db, dl, tuning=tu(mode), codes_misalign=mis)


# --------------------------------------------------------------------------- #
# slices, alignment, empty and degenerate columns
# --------------------------------------------------------------------------- #
@pytest.mark.parametrize("mis", [1, 3, 8, 15])
def test_misaligned_pointers_fsst(datagen_mod, mis):
    c = datagen_mod.fsst_small(seed=9, n_strings=1500)
    assert_parity("fsst8", c.codes, c.code_off, c.dict_bytes, c.dict_lens, codes_misalign=mis, out_misalign=mis)


@pytest.mark.parametrize("mis", [2, 6, 14])
def test_misaligned_pointers_onpair(datagen_mod, mis):
    c = datagen_mod.onpair_urls(seed=10, target_bytes=256 << 10, sample_bytes=512 << 10)
    assert_parity("onpair16", c.codes, c.code_off, c.dict_bytes, c.dict_lens, codes_misalign=mis,
                  out_misalign=mis + 1)


def test_slice(datagen_mod):
    """code_offsets[0] > 0 and code_offsets[-1] < n_codes (an Arrow slice)."""
    c = datagen_mod.fsst_small(seed=12, n_strings=4000)
    sl = c.code_off[1000:3001].astype(np.int64)
    assert_parity("fsst8", c.codes, sl, c.dict_bytes, c.dict_lens)
    c2 = datagen_mod.onpair_urls(seed=13, target_bytes=512 << 10, sample_bytes=512 << 10)
    sl2 = c2.code_off[777:5555]
    assert_parity("onpair16", c2.codes, sl2, c2.dict_bytes, c2.dict_lens)


def test_empty_and_degenerate():
    db, dl = pack([b"ab", b"c"])
    u8 = lambda *x: np.array(x, np.uint8)
    # no strings
    assert_parity("fsst8", u8(0, 1), np.array([0], np.int64), db, dl)
    assert_parity("fsst8", np.zeros(0, np.uint8), np.array([0], np.int32), db, dl)
    # all strings empty
    assert_parity("fsst8", u8(0, 1, 1), np.zeros(1000, np.int64), db, dl)
    # one code
    assert_parity("fsst8", u8(1), np.array([0, 1], np.int64), db, dl)
    assert_parity("onpair16", np.array([1], np.uint16), np.array([0, 1], np.int64), db, dl)
    # strings of a single escape pair; empty strings in between
    assert_parity("fsst8", u8(255, 7, 255, 255), np.array([0, 2, 2, 2, 4], np.int64), db, dl)
    # empty dictionary: every code is bad
    assert_parity("fsst8", u8(0), np.array([0, 1], np.int64), np.zeros(0, np.uint8), np.zeros(0, np.uint8),
                  via="oneshot")


@pytest.mark.parametrize("case", ["identity_onpair", "identity_fsst"])
def test_identity_dictionaries(case):
    rng = np.random.default_rng(3)
    if case == "identity_onpair":
        db, dl = pack([bytes([b]) for b in range(256)])
        codes = rng.integers(0, 256, size=300_000).astype(np.uint16)
        off = np.concatenate([[0], np.sort(rng.integers(0, len(codes), 4999)), [len(codes)]]).astype(np.int64)
        exp = assert_parity("onpair16", codes, off, db, dl)
        assert np.array_equal(exp.out_bytes, codes.astype(np.uint8))
    else:
        db, dl = pack([bytes([b]) for b in range(255)])
        text = rng.integers(0, 256, size=200_000).astype(np.uint8)
        codes = np.frombuffer(text.tobytes().replace(b"\xff", b"\xff\xff"), np.uint8).copy()
        exp = assert_parity("fsst8", codes, np.array([0, len(codes)], np.int64), db, dl)
        assert np.array_equal(exp.out_bytes, text)


# --------------------------------------------------------------------------- #
# errors (device-detected) and the status protocol
# --------------------------------------------------------------------------- #
def test_device_errors():
    db, dl = pack([b"ab", b"c"])
    u8 = lambda *x: np.array(x, np.uint8)
    i64 = lambda *x: np.array(x, np.int64)
    assert_parity("fsst8", u8(0, 9, 1), i64(0, 3), db, dl)                 # EBADCODE
    assert_parity("fsst8", u8(0, 255, 1), i64(0, 2, 3), db, dl)            # EESCAPE (escape ends string 0)
    assert_parity("fsst8", u8(0, 1, 255, 255, 255), i64(0, 2, 5), db, dl)  # EESCAPE after a literal 255
    assert_parity("fsst8", u8(0, 1, 0), i64(0, 2, 1), db, dl)              # EOFFSETS (decreasing)
    assert_parity("fsst8", u8(0, 1, 0), i64(-1, 2), db, dl)                # EOFFSETS (negative)
    assert_parity("fsst8", u8(0, 1, 0), i64(0, 4), db, dl)                 # EOFFSETS (past n_codes)
    assert_parity("fsst8", u8(0, 1), i64(0, 2), *pack([b"", b"c"]), via="oneshot")   # EBADDICT
    assert_parity("fsst8", u8(0, 1), i64(0, 2), *pack([b"123456789", b"c"]), via="oneshot")
    assert_parity("onpair16", np.array([0, 5], np.uint16), i64(0, 2), db, dl)   # EBADCODE
    assert_parity("onpair16", np.array([0, 1], np.uint16), i64(0, 2), *pack([b"x" * 17, b"c"]), via="oneshot")
    # precedence: the data error at the lowest position wins
    assert_parity("fsst8", u8(9, 0, 255), i64(0, 3), db, dl)
    assert_parity("fsst8", u8(0, 255, 9), i64(0, 2, 3), db, dl)
    # EBADDICT before EOFFSETS before data errors
    assert_parity("fsst8", u8(9), i64(1, 0), *pack([b"", b"c"]), via="oneshot")
    assert_parity("fsst8", u8(9), i64(0, 2), db, dl)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("bad_at", [None, 3, 200_000])
def test_onpair16_short_dictionary_many_tiles(datagen_mod, mode, bad_at):
    """OnPair-16 over many tiles with a 1,000-token dictionary; with bad_at a
    code past the dictionary (and a token of 16 bytes elsewhere): the status is
    the oracle's, and without one the output is, in both ways to the cursors."""
    c = datagen_mod.random_onpair(seed=41, n_codes=300_000, n_strings=20_000, n_tok=1000)
    codes = c.codes.copy()
    dl = c.dict_lens.copy()
    assert (dl == 16).any()
    if bad_at is not None:
        codes[bad_at] = 1000 + bad_at % 7
    for tc in (0, 64):
        assert_parity("onpair16", codes, c.code_off, c.dict_bytes, dl, tuning=tu(mode, tc))


def test_dict_create_rejects_bad_lengths():
    import torch
    import paper_2609_15034_amd as fd
    for codec, toks in (("fsst8", [b"", b"a"]), ("fsst8", [b"123456789"]), ("onpair16", [b"x" * 17]),
                        ("onpair16", [b"a", b""])):
        db, dl = pack(toks)
        dbt = torch.from_numpy(db if len(db) else np.zeros(1, np.uint8)).cuda()
        with pytest.raises(fd.DecodeError) as e:
            fd.Dict(codec, dbt, torch.from_numpy(dl).cuda())
        assert e.value.status == fd.EBADDICT


def test_capacity_too_small(datagen_mod):
    """ECAPACITY: offsets complete, bytes below the capacity correct, nothing
    written past it (guard bands)."""
    c = datagen_mod.fsst_small(seed=21, n_strings=2000)
    total = len(c.text)
    for cap in (0, 1, 17, total // 2, total - 1):
        assert_parity("fsst8", c.codes, c.code_off, c.dict_bytes, c.dict_lens, cap=cap)
    assert_parity("fsst8", c.codes, c.code_off, c.dict_bytes, c.dict_lens, cap=total)
    c2 = datagen_mod.onpair_urls(seed=22, target_bytes=256 << 10, sample_bytes=256 << 10)
    assert_parity("onpair16", c2.codes, c2.code_off, c2.dict_bytes, c2.dict_lens, cap=len(c2.text) // 3)


def test_overflow_int32():
    """int32 offsets cannot hold 2**31 decoded bytes: EOVERFLOW (capacity 0,
    so no 2 GiB output is needed), and exactly INT32_MAX fits."""
    db, dl = pack([b"0123456789abcdef", b"0123456789abcde"])
    n = 2 ** 27
    codes = np.zeros(n, np.uint16)
    st, _, _, _ = gpu_decode("onpair16", codes, np.array([0, n], np.int32), db, dl, cap=0)
    assert st == 5
    codes[-1] = 1
    st, off, _, _ = gpu_decode("onpair16", codes, np.array([0, n], np.int32), db, dl, cap=0)
    assert st == 4 and int(off[-1]) == 2 ** 31 - 1


def test_async_status(datagen_mod):
    c = datagen_mod.fsst_small(seed=31, n_strings=500)
    assert_parity("fsst8", c.codes, c.code_off, c.dict_bytes, c.dict_lens, async_=True)
    db, dl = pack([b"ab", b"c"])
    assert_parity("fsst8", np.array([0, 9], np.uint8), np.array([0, 2], np.int64), db, dl, async_=True)


def test_determinism_repeated(datagen_mod):
    """Tiny tiles (long look-back chains) and different grids: every repeat is
    identical to the oracle."""
    c = datagen_mod.fsst_small(seed=41, n_strings=4000)
    for rep in range(12):
        grid = [0, 1, 3, 64][rep % 4]
        assert_parity("fsst8", c.codes, c.code_off, c.dict_bytes, c.dict_lens, tuning=tu(0, 16 * (1 + rep % 3), grid))


def test_decode_convenience(datagen_mod):
    import torch
    import oracle
    import paper_2609_15034_amd as fd
    c = datagen_mod.onpair_urls(seed=51, target_bytes=512 << 10, sample_bytes=512 << 10)
    d = fd.Dict("onpair16", torch.from_numpy(c.dict_bytes).cuda(), torch.from_numpy(c.dict_lens).cuda())
    off, out = fd.decode(d, torch.from_numpy(c.codes.view(np.int16)).cuda(), torch.from_numpy(c.code_off).cuda())
    exp = oracle.decode("onpair16", c.codes, c.code_off, c.dict_bytes, c.dict_lens)
    assert np.array_equal(off.cpu().numpy(), exp.out_off) and np.array_equal(out.cpu().numpy(), exp.out_bytes)


# --------------------------------------------------------------------------- #
# tiles at fixed code positions: slices, strings across many tiles, runs of
# empty strings, offsets that are wrong anywhere
# --------------------------------------------------------------------------- #
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("tc", [0, 16, 48])
def test_slice_small_tiles(datagen_mod, mode, tc):
    """A slice: tiles are positions of the whole buffer, so the first and last
    tiles hold part of the range and tiles before it hold nothing."""
    c = datagen_mod.fsst_small(seed=12, n_strings=4000)
    sl = c.code_off[1000:3001].astype(np.int64)
    assert_parity("fsst8", c.codes, sl, c.dict_bytes, c.dict_lens, tuning=tu(mode, tc))
    c2 = datagen_mod.onpair_urls(seed=13, target_bytes=512 << 10, sample_bytes=512 << 10)
    sl2 = c2.code_off[777:5555]
    assert_parity("onpair16", c2.codes, sl2, c2.dict_bytes, c2.dict_lens, tuning=tu(mode, tc))


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("tc", [0, 16])
def test_string_across_many_tiles(mode, tc):
    """One string of 300,000 codes among short ones: 18,750 tiles of 16 codes
    own no string start (the coarse index writes them in one wave's loop)."""
    rng = np.random.default_rng(61)
    db, dl = pack([b"a", b"bc", b"def", b"\xff\x00"])
    lens = [3, 0, 300_000, 5, 0, 0, 7, 1]
    codes = rng.integers(0, 4, size=sum(lens)).astype(np.uint8)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    assert_parity("fsst8", codes, off, db, dl, tuning=tu(mode, tc))
    assert_parity("onpair16", codes.astype(np.uint16), off, db, dl, tuning=tu(mode, 8 if tc else 0))


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("tc", [0, 16])
def test_runs_of_empty_strings(mode, tc):
    """Tens of thousands of empty strings at a few positions (a tile owning
    many strings reads its code offsets in several steps), also at both ends."""
    db, dl = pack([b"a", b"bc", b"def"])
    rng = np.random.default_rng(62)
    codes = rng.integers(0, 3, size=5000).astype(np.uint8)
    pos = np.sort(np.concatenate([np.zeros(20_000), np.full(30_000, 2500), rng.integers(0, 5001, 3000),
                                  np.full(10_000, 5000)])).astype(np.int64)
    off = np.concatenate([[0], pos, [5000]]).astype(np.int64)
    assert_parity("fsst8", codes, off, db, dl, tuning=tu(mode, tc))


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("tc", [0, 16, 160])
def test_bad_offsets_anywhere(datagen_mod, mode, tc):
    """A code offset that breaks the order anywhere is found, whichever tile
    reads it: a too large or a too small entry at random places."""
    c = datagen_mod.fsst_small(seed=63, n_strings=3000)
    rng = np.random.default_rng(64)
    for k in range(12):
        off = c.code_off.astype(np.int64).copy()
        i = int(rng.integers(1, len(off) - 1))
        off[i] = off[i + 1] + 1 + int(rng.integers(0, 50)) if k % 2 == 0 else max(0, off[i - 1] - 1 - int(
            rng.integers(0, 50)))
        if np.all(np.diff(off) >= 0):
            continue
        assert_parity("fsst8", c.codes, off, c.dict_bytes, c.dict_lens, tuning=tu(mode, tc))


# --------------------------------------------------------------------------- #
# tiles whose output spans several staging windows (long tokens at full tile
# sizes), next to tiles of one window, with escapes
# --------------------------------------------------------------------------- #
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("long_share", [1.0, 0.5])
def test_fsst_multi_window_tiles(mode, long_share):
    """254 eight-byte symbols and code 254 of one byte: at the full tile of
    8,176 codes a tile decodes to up to 64 KiB, several 16 KiB windows;
    long_share < 1 mixes in short codes and escapes, so neighbouring tiles
    take one window or several."""
    rng = np.random.default_rng(int(long_share * 10) + 17 * mode)
    syms = [bytes(rng.integers(0, 256, 8, dtype=np.uint8)) for _ in range(254)] + [b"\x07"]
    db, dl = pack(syms)
    n = 300_000
    codes = rng.integers(0, 254, n).astype(np.uint8)
    short = rng.random(n) > long_share
    codes[short] = 254
    esc = np.flatnonzero(rng.random(n - 1) < 0.02 * (1.0 - long_share))
    codes[esc] = 255                               # an escape; its literal is the next byte
    cuts = np.sort(rng.choice(np.arange(1, n), 2000, replace=False))
    codes[cuts - 1] = 254                          # no string ends on an escape
    codes[-1] = 254
    code_off = np.concatenate([[0], cuts, [n]]).astype(np.int64)
    exp = assert_parity("fsst8", codes, code_off, db, dl, tuning=tu(mode))
    assert exp.status == 0


@pytest.mark.parametrize("mode", [0, 1])
def test_onpair_multi_window_tiles(mode):
    """Sixteen-byte tokens: a full OnPair tile of 4,088 codes decodes to 64
    KiB, two or three 32 KiB windows; one-byte tokens in half the tiles'
    stretches give tiles of one window next to them."""
    rng = np.random.default_rng(23 + mode)
    toks = [bytes(rng.integers(0, 256, 16, dtype=np.uint8)) for _ in range(1000)] + [bytes([b]) for b in range(256)]
    db, dl = pack(toks)
    n = 200_000
    codes = rng.integers(0, 1000, n).astype(np.uint16)
    stretch = (np.arange(n) // 3000) % 2 == 1
    codes[stretch] = 1000 + rng.integers(0, 256, int(stretch.sum())).astype(np.uint16)
    cuts = np.sort(rng.choice(np.arange(1, n), 5000, replace=False))
    code_off = np.concatenate([[0], cuts, [n]]).astype(np.int64)
    exp = assert_parity("onpair16", codes, code_off, db, dl, tuning=tu(mode))
    assert exp.status == 0


def test_automatic_mode_both_sides(datagen_mod):
    """Without a tuning the decode picks the three phases for a column with at
    least four times as many tiles as resident workgroups (a 96 MiB log column
    has about 7,000 tiles of 8,176 codes, against 4 x 5 x 256) and the single
    pass for a small one (the profiler sees a totals launch only in the
    former); both match the oracle."""
    import paper_2609_15034_amd as fd
    big = datagen_mod.fsst_logs(seed=41, target_bytes=96 << 20)
    assert len(big.codes) // 8176 >= 4 * 5 * 256
    small = datagen_mod.fsst_small(seed=42)
    for c, three in ((big, True), (small, False)):
        fd.profile_begin(("totals", "decode"), 64)
        exp = assert_parity("fsst8", c.codes, c.code_off, c.dict_bytes, c.dict_lens)
        pr = fd.profile_end()
        assert ("totals" in pr) == three, pr
        assert np.array_equal(exp.out_bytes, c.text)
