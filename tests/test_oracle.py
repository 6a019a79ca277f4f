"""Pins for the CPU oracle (no GPU).

The paper prints no worked input/output example, so the oracle is pinned by
checks that do not restate its loop:
  * round trips through independent greedy longest-match encoders
    (decode(encode(text)) == text) on every workload recipe;
  * a closed-form characterisation of FSST-8 escapes (a position is a literal
    iff the run of 255s right before it in its string has odd length),
    evaluated exhaustively on short code strings;
  * brute force of token concatenation against ``b"".join``;
  * identity dictionaries (decode reduces to a cast / an unescape);
  * the copy-16-and-advance CPU loop described for OnPair;
  * hand-derived cases under tests/golden/;
  * error precedence on constructed malformed inputs.
"""
import itertools

import numpy as np
import pytest

from conftest import parse_golden

# --------------------------------------------------------------------------- #
# helpers independent of the oracle
# --------------------------------------------------------------------------- #


def closed_form_fsst8(codes: bytes, code_off, syms):
    """Expected (status, out_off, out) from the run-parity characterisation:
    position p is a literal iff the run of consecutive 255 bytes immediately
    before p (within its string) has odd length; a 255 that is not a literal is
    an escape; any other position is a code.  Errors in stream order."""
    out = bytearray()
    offs = [0]
    for i in range(len(code_off) - 1):
        a, e = code_off[i], code_off[i + 1]
        for p in range(a, e):
            run = 0
            q = p - 1
            while q >= a and codes[q] == 255:
                run += 1
                q -= 1
            literal = run % 2 == 1
            if literal:
                out.append(codes[p])
            elif codes[p] == 255:
                if p == e - 1:
                    return 3, None, None
            else:
                if codes[p] >= len(syms):
                    return 2, None, None
                out += syms[codes[p]]
        offs.append(len(out))
    return 0, offs, bytes(out)


def pack(tokens):
    lens = np.array([len(t) for t in tokens], np.uint8)
    return np.frombuffer(b"".join(tokens), np.uint8).copy(), lens


# --------------------------------------------------------------------------- #
# round trips on every recipe
# --------------------------------------------------------------------------- #


def test_roundtrip_fsst_small(oracle_mod, datagen_mod):
    c = datagen_mod.fsst_small()
    assert c.code_off.dtype == np.int32
    assert 0.01 <= c.stats["escape_share"] <= 0.03
    r = oracle_mod.decode("fsst8", c.codes, c.code_off, c.dict_bytes, c.dict_lens)
    assert r.status == 0
    assert np.array_equal(r.out_off, c.text_off)
    assert np.array_equal(r.out_bytes, c.text)


def test_roundtrip_fsst_logs(oracle_mod, datagen_mod):
    c = datagen_mod.fsst_logs(target_bytes=4 << 20, sample_bytes=1 << 20)
    assert c.stats["n_escapes"] > 0
    r = oracle_mod.decode("fsst8", c.codes, c.code_off, c.dict_bytes, c.dict_lens)
    assert r.status == 0
    assert np.array_equal(r.out_off, c.text_off)
    assert np.array_equal(r.out_bytes, c.text)


def test_roundtrip_onpair_urls(oracle_mod, datagen_mod):
    c = datagen_mod.onpair_urls(target_bytes=4 << 20, sample_bytes=1 << 20)
    assert len(c.dict_lens) > 256 and c.dict_lens.max() <= 16
    r = oracle_mod.decode("onpair16", c.codes, c.code_off, c.dict_bytes, c.dict_lens)
    assert r.status == 0
    assert np.array_equal(r.out_off, c.text_off)
    assert np.array_equal(r.out_bytes, c.text)
    # the copy-16-and-advance formulation agrees
    st, off2, out2 = oracle_mod.decode_onpair16_copy16(c.codes, c.code_off, c.dict_bytes, c.dict_lens)
    assert st == 0 and np.array_equal(off2, r.out_off) and np.array_equal(out2, r.out_bytes)


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_roundtrip_ff_heavy(oracle_mod, datagen_mod, seed):
    """Strings over {0x00, 'a', 0xFF} with a table that lacks 0xFF: every 0xFF is
    stored as escape + literal 0xFF, giving long 255 runs."""
    rng = np.random.default_rng(seed)
    alphabet = np.array([0x00, 0x61, 0xFF], np.uint8)
    lens = rng.integers(0, 40, size=300)
    text = alphabet[rng.integers(0, 3, size=int(lens.sum()))]
    toff = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    tokens = [b"\x00", b"a", b"aa", b"a\x00", b"\x00\x00\x00"]
    db, dl = pack(tokens)
    codes, coff, esc = datagen_mod.encode_fsst(db, dl, text, toff)
    assert esc == int((text == 0xFF).sum())
    r = oracle_mod.decode("fsst8", codes, coff, db, dl)
    assert r.status == 0
    assert np.array_equal(r.out_off, toff) and np.array_equal(r.out_bytes, text)


def test_roundtrip_random_tables(oracle_mod, datagen_mod):
    """Random byte strings (all 256 values) under random FSST and OnPair tables."""
    rng = np.random.default_rng(5)
    lens = rng.integers(0, 64, size=500)
    text = rng.integers(0, 256, size=int(lens.sum())).astype(np.uint8)
    toff = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    db, dl = datagen_mod.random_dict(21, n_tok=255, max_len=8)
    codes, coff, _ = datagen_mod.encode_fsst(db, dl, text, toff)
    r = oracle_mod.decode("fsst8", codes, coff, db, dl)
    assert r.status == 0 and np.array_equal(r.out_bytes, text) and np.array_equal(r.out_off, toff)
    # OnPair: 256 single bytes + random longer tokens
    singles = [bytes([b]) for b in range(256)]
    rb, rl = datagen_mod.random_dict(22, n_tok=4000, max_len=16)
    extra, pos = [], 0
    for l in rl.tolist():
        extra.append(bytes(rb[pos:pos + l]))
        pos += l
    db2, dl2 = pack(singles + extra)
    codes2, coff2, _ = datagen_mod.encode_onpair(db2, dl2, text, toff)
    r2 = oracle_mod.decode("onpair16", codes2, coff2, db2, dl2)
    assert r2.status == 0 and np.array_equal(r2.out_bytes, text) and np.array_equal(r2.out_off, toff)


# --------------------------------------------------------------------------- #
# escape logic: closed form + pure-Python transcription, exhaustive
# --------------------------------------------------------------------------- #


def test_escape_closed_form_exhaustive(oracle_mod):
    from oracle import spec
    syms = [b"AB", b"c"]                       # codes 0, 1 valid; 254 and 'x' are bad unless literal
    db, dl = pack(syms)
    alphabet = [0, 1, 254, 255, ord("x")]
    n_cases = 0
    for L in range(0, 7):
        for combo in itertools.product(alphabet, repeat=L):
            codes = bytes(combo)
            coff = [0, L]
            exp = closed_form_fsst8(codes, coff, syms)
            r = oracle_mod.decode("fsst8", np.frombuffer(codes, np.uint8) if L else np.zeros(0, np.uint8),
                                  np.array(coff, np.int64), db, dl)
            assert r.status == exp[0], (codes, r.status, exp[0])
            sp = spec.decode_fsst8(codes, coff, syms)
            assert sp[0] == exp[0]
            if exp[0] == 0:
                assert list(r.out_off) == exp[1] and bytes(r.out_bytes) == exp[2], codes
                assert sp[1] == exp[1] and sp[2] == exp[2]
            n_cases += 1
    assert n_cases == sum(5 ** L for L in range(7))


def test_escape_closed_form_multistring_random(oracle_mod):
    """Many strings in one column, long 255 runs crossing string boundaries."""
    rng = np.random.default_rng(3)
    syms = [b"p", b"qq", b"rrr"]
    db, dl = pack(syms)
    for trial in range(200):
        n = int(rng.integers(1, 12))
        parts = []
        for _ in range(n):
            L = int(rng.integers(0, 12))
            # valid strings: units are codes 0..2 or (255, any byte)
            s = bytearray()
            while len(s) < L:
                if rng.random() < 0.5:
                    s += bytes([255, int(rng.choice([255, 0, 7, 200]))])
                else:
                    s.append(int(rng.integers(0, 3)))
            parts.append(bytes(s))
        codes = b"".join(parts)
        coff = [0] + list(np.cumsum([len(p) for p in parts]))
        exp = closed_form_fsst8(codes, coff, syms)
        assert exp[0] == 0
        r = oracle_mod.decode("fsst8", np.frombuffer(codes, np.uint8) if codes else np.zeros(0, np.uint8),
                              np.array(coff, np.int64), db, dl)
        assert r.status == 0 and list(r.out_off) == exp[1] and bytes(r.out_bytes) == exp[2]


# --------------------------------------------------------------------------- #
# token concatenation, brute force
# --------------------------------------------------------------------------- #


def test_token_concat_bruteforce(oracle_mod):
    rng = np.random.default_rng(9)
    toks = [bytes(rng.integers(0, 256, size=l).astype(np.uint8)) for l in (1, 7, 8, 9, 15, 16)]
    db, dl = pack(toks)
    seqs = [s for L in range(0, 5) for s in itertools.product(range(6), repeat=L)]
    codes = np.array([c for s in seqs for c in s], np.uint16)
    coff = np.concatenate([[0], np.cumsum([len(s) for s in seqs])]).astype(np.int64)
    r = oracle_mod.decode("onpair16", codes, coff, db, dl)
    assert r.status == 0
    expect = [b"".join(toks[c] for c in s) for s in seqs]
    assert list(np.diff(r.out_off)) == [len(e) for e in expect]
    assert bytes(r.out_bytes) == b"".join(expect)


# --------------------------------------------------------------------------- #
# identity dictionaries
# --------------------------------------------------------------------------- #


def test_identity_onpair(oracle_mod):
    db, dl = pack([bytes([b]) for b in range(256)])
    rng = np.random.default_rng(1)
    codes = rng.integers(0, 256, size=100_000).astype(np.uint16)
    coff = np.concatenate([[0], np.sort(rng.integers(0, len(codes), size=999)), [len(codes)]]).astype(np.int64)
    r = oracle_mod.decode("onpair16", codes, coff, db, dl)
    assert r.status == 0
    assert np.array_equal(r.out_bytes, codes.astype(np.uint8))
    assert np.array_equal(r.out_off, coff - coff[0])


def test_identity_fsst(oracle_mod):
    db, dl = pack([bytes([b]) for b in range(255)])
    rng = np.random.default_rng(2)
    text = rng.integers(0, 256, size=50_000).astype(np.uint8)
    # escape every 0xFF: codes = text with each 0xFF replaced by (255, 255)
    codes = bytearray()
    for b in text.tobytes():
        codes += b"\xff\xff" if b == 255 else bytes([b])
    r = oracle_mod.decode("fsst8", np.frombuffer(bytes(codes), np.uint8), np.array([0, len(codes)], np.int64),
                          db, dl)
    assert r.status == 0 and np.array_equal(r.out_bytes, text)
    # unescaping the codes (a 255 consumes the next byte) gives the text back too
    un, i = bytearray(), 0
    while i < len(codes):
        if codes[i] == 255:
            un.append(codes[i + 1])
            i += 2
        else:
            un.append(codes[i])
            i += 1
    assert bytes(un) == bytes(r.out_bytes)


def test_offsets_closed_form_total(oracle_mod, datagen_mod):
    """total = sum of token lengths of non-escape codes + number of literals,
    and per-string lengths match the per-string sums."""
    c = datagen_mod.fsst_small(seed=7, n_strings=2000)
    r = oracle_mod.decode("fsst8", c.codes, c.code_off, c.dict_bytes, c.dict_lens)
    assert r.status == 0
    assert np.all(np.diff(r.out_off) >= 0)
    codes = c.codes.tobytes()
    lens = [int(x) for x in c.dict_lens]
    tot = 0
    for i in range(c.n_strings):
        a, e = int(c.code_off[i]), int(c.code_off[i + 1])
        s, p = 0, a
        while p < e:
            if codes[p] == 255:
                s += 1
                p += 2
            else:
                s += lens[codes[p]]
                p += 1
        assert r.out_off[i + 1] - r.out_off[i] == s
        tot += s
    assert r.total == tot == len(c.text)


# --------------------------------------------------------------------------- #
# golden hand-derived cases
# --------------------------------------------------------------------------- #


@pytest.mark.parametrize("case", parse_golden("fsst8_cases.txt"), ids=lambda c: c["line"][:40])
def test_golden_fsst8(oracle_mod, case):
    codes = bytes.fromhex("".join(case["codes"]))
    db, dl = pack(case["tokens"])
    r = oracle_mod.decode("fsst8", np.frombuffer(codes, np.uint8) if codes else np.zeros(0, np.uint8),
                          np.array(case["code_off"], np.int64), db, dl)
    assert r.status == case["status"]
    if case["out_off"] is not None:
        assert list(r.out_off) == case["out_off"]
        assert bytes(r.out_bytes) == case["bytes"]


@pytest.mark.parametrize("case", parse_golden("onpair16_cases.txt"), ids=lambda c: c["line"][:40])
def test_golden_onpair16(oracle_mod, case):
    codes = np.array([int(x) for x in case["codes"]], np.uint16)
    db, dl = pack(case["tokens"])
    r = oracle_mod.decode("onpair16", codes, np.array(case["code_off"], np.int64), db, dl)
    assert r.status == case["status"]
    if case["out_off"] is not None:
        assert list(r.out_off) == case["out_off"]
        assert bytes(r.out_bytes) == case["bytes"]


@pytest.mark.parametrize("case", parse_golden("code12_cases.txt"), ids=lambda c: c["line"][:40])
def test_golden_code12(oracle_mod, case):
    packed = np.frombuffer(bytes.fromhex("".join(case["codes"])), np.uint8)
    db, dl = pack(case["tokens"])
    r = oracle_mod.decode("onpair12", packed, np.array(case["code_off"], np.int64), db, dl)
    assert r.status == case["status"]
    if case["out_off"] is not None:
        assert list(r.out_off) == case["out_off"]
        assert bytes(r.out_bytes) == case["bytes"]


def test_unpack12_by_hand(oracle_mod):
    """Bit order of the 12-bit stream, values worked out by hand."""
    assert oracle_mod.unpack12(np.array([0x23, 0xC1, 0xAB], np.uint8), 2).tolist() == [0x123, 0xABC]
    assert oracle_mod.unpack12(np.array([0xFF, 0x0F, 0x00, 0x01, 0x0F], np.uint8), 3).tolist() == [0xFFF, 0x000, 0xF01]
    # every 12-bit value at both phases (even and odd code positions)
    v = np.arange(4096)
    for shift in (0, 1):
        codes = np.concatenate([np.zeros(shift, np.int64), v])
        assert np.array_equal(oracle_mod.unpack12(oracle_mod.pack12(codes), len(codes))[shift:], v)


def test_unpack12_whole_column_form(oracle_mod):
    """The vectorised unpacker the oracle uses on whole columns agrees with the
    one-code-at-a-time definition."""
    rng = np.random.default_rng(12)
    for n in (0, 1, 2, 3, 1000, 1001):
        packed = rng.integers(0, 256, (n * 12 + 7) // 8).astype(np.uint8)
        assert np.array_equal(oracle_mod.unpack12_np(packed, n), oracle_mod.unpack12(packed, n))


def test_roundtrip_code12(oracle_mod, datagen_mod):
    """OnPair-12 and FSST-12 columns decode back to their source text."""
    for col in (datagen_mod.onpair12_urls(target_bytes=1 << 19), datagen_mod.fsst12_logs(target_bytes=1 << 19)):
        r = oracle_mod.decode("onpair12", col.codes, col.code_off, col.dict_bytes, col.dict_lens,
                              n_codes=col.stats["n_codes"])
        assert r.status == 0
        assert np.array_equal(r.out_bytes, col.text) and np.array_equal(r.out_off, col.text_off)
        assert len(col.dict_lens) <= 4096


# --------------------------------------------------------------------------- #
# the sidecar (stored output positions per tile of strings)
# --------------------------------------------------------------------------- #


def tile_starts(n_codes, a, b, T):
    """The code position of every tile's first code, then the end b."""
    n_tiles = max(1, -(-n_codes // T))
    return [max(a, min(k * T, b)) for k in range(n_tiles)] + [b]


def test_sidecar_by_hand(oracle_mod):
    """Positions derived by hand.  FSST-8 table {0: "ab", 1: "c"}; strings
    "abc" (codes 0 1), "x" (escape + literal), "ab" (0), "" and "cc" (1 1):
    code positions 0..7 start at output bytes 0, 2, 3, 3, 4, 6, 7, 8 (the
    escape at 2 emits nothing, its literal at 3 one byte).  OnPair-16 tokens
    {"a", "bcd", "ef"}; codes 1 2 | 0 | 2 2 1 (lengths 3 2 1 2 2 3): code
    positions start at 0, 3, 5, 6, 8, 10, 13."""
    O = oracle_mod
    db, dl = pack([b"ab", b"c"])
    codes = np.array([0, 1, 255, ord("x"), 0, 1, 1], np.uint8)
    off = np.array([0, 2, 4, 5, 5, 7], np.int64)
    for T, exp in ((1, [0, 2, 3, 3, 4, 6, 7, 8]), (2, [0, 3, 4, 7, 8]), (3, [0, 3, 7, 8]), (16, [0, 8])):
        st, sc = O.sidecar("fsst8", codes, off, db, dl, T)
        assert st == O.OK and list(sc) == exp, T
    db2, dl2 = pack([b"a", b"bcd", b"ef"])
    st, sc = O.sidecar("onpair16", np.array([1, 2, 0, 2, 2, 1], np.uint16), np.array([0, 2, 3, 6], np.int64),
                       db2, dl2, 2)
    assert st == O.OK and list(sc) == [0, 5, 8, 13]
    # a slice: the decode range [2, 6) of the same codes (the strings 0 | 2 2 1... from position 2)
    st, sc = O.sidecar("onpair16", np.array([1, 2, 0, 2, 2, 1], np.uint16), np.array([2, 3, 6], np.int64),
                       db2, dl2, 4)
    assert st == O.OK and list(sc) == [0, 3, 8]
    # a tile boundary right after an escape: position 3 is the literal
    st, sc = O.sidecar("fsst8", codes, off, db, dl, 3)
    assert list(sc)[1] == 3
    # no strings: one empty tile
    st, sc = O.sidecar("fsst8", np.zeros(0, np.uint8), np.array([0], np.int64), db[:1], dl[:1], 4)
    assert st == O.OK and list(sc) == [0, 0]


@pytest.mark.parametrize("T", [16, 48, 1000, 4088])
def test_sidecar_at_string_starts_is_the_source_offsets(oracle_mod, datagen_mod, T):
    """Decoding is lossless, so where a tile starts exactly at a string, the
    stored position is that source string's own offset (the generator's
    offsets, not a decode); every entry is non-decreasing and the last is the
    total of the source text."""
    cols = [(datagen_mod.fsst_small(), "fsst8", None),
            (datagen_mod.onpair_urls(target_bytes=1 << 20, sample_bytes=1 << 20), "onpair16", None)]
    c12 = datagen_mod.onpair12_urls(target_bytes=1 << 19)
    cols.append((c12, "onpair12", c12.stats["n_codes"]))
    for c, codec, n_codes in cols:
        nc = len(c.codes) if n_codes is None else n_codes
        st, sc = oracle_mod.sidecar(codec, c.codes, c.code_off, c.dict_bytes, c.dict_lens, T, n_codes=n_codes)
        assert st == 0
        co = np.asarray(c.code_off, np.int64)
        pos = tile_starts(nc, int(co[0]), int(co[-1]), T)
        hits = 0
        for k, p in enumerate(pos):
            i = np.searchsorted(co, p, side="right") - 1
            if co[i] == p:                            # a string starts here (the last of any empty ones)
                assert sc[k] == c.text_off[i], (codec, k)
                hits += 1
        assert hits >= 2
        assert np.all(np.diff(sc) >= 0) and sc[-1] == len(c.text)


def test_sidecar_onpair_cumulative_lengths(oracle_mod, datagen_mod):
    """OnPair has no escapes: the position of code p is the sum of the token
    lengths of the codes before it (a cumulative sum, another formulation)."""
    c = datagen_mod.onpair_urls(target_bytes=1 << 20, sample_bytes=1 << 20)
    cum = np.concatenate([[0], np.cumsum(c.dict_lens[c.codes].astype(np.int64))])
    co = np.asarray(c.code_off, np.int64)
    for T in (8, 200, 4088):
        st, sc = oracle_mod.sidecar("onpair16", c.codes, c.code_off, c.dict_bytes, c.dict_lens, T)
        pos = tile_starts(len(c.codes), int(co[0]), int(co[-1]), T)
        assert st == 0 and np.array_equal(sc, cum[pos] - cum[co[0]])


def test_sidecar_escape_closed_form(oracle_mod):
    """With escapes, against the run-parity characterisation: every code's
    length (1 for a literal, 0 for an escape, else its symbol's) summed up to
    each tile start."""
    rng = np.random.default_rng(5)
    syms = [bytes(rng.integers(97, 123, int(k)).astype(np.uint8)) for k in rng.integers(1, 9, 200)]
    db, dl = pack(syms)
    n = 300
    lens = rng.integers(0, 12, n)
    code_off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    pool = np.array(list(range(200)) + [255] * 60, np.uint8)
    codes = pool[rng.integers(0, len(pool), int(code_off[-1]))]
    for i in range(n):                         # no string ends in an unpaired escape
        a, e = int(code_off[i]), int(code_off[i + 1])
        if e > a and codes[e - 1] == 255:
            codes[e - 1] = 7
    st, offs, _ = closed_form_fsst8(codes.tobytes(), [int(x) for x in code_off], syms)
    if st != 0:
        pytest.skip("the random stream ended a string in an escape run")
    per = np.zeros(len(codes), np.int64)
    for i in range(n):
        a, e = int(code_off[i]), int(code_off[i + 1])
        for p in range(a, e):
            run, q = 0, p - 1
            while q >= a and codes[q] == 255:
                run, q = run + 1, q - 1
            per[p] = 1 if run % 2 else (0 if codes[p] == 255 else len(syms[codes[p]]))
    cum = np.concatenate([[0], np.cumsum(per)])
    assert cum[-1] == offs[-1]
    for T in (1, 7, 16, 64):
        st2, sc = oracle_mod.sidecar("fsst8", codes, code_off, db, dl, T)
        assert st2 == 0 and np.array_equal(sc, cum[tile_starts(len(codes), 0, len(codes), T)]), T


def test_decode_with_sidecar_precedence(oracle_mod):
    """A matching sidecar gives the plain decode; any other gives ESIDECAR,
    after the errors in the data and before EOVERFLOW / ECAPACITY."""
    O = oracle_mod
    db, dl = pack([b"ab", b"c"])
    codes = np.array([0, 1, 255, ord("x"), 0, 1, 1], np.uint8)
    off = np.array([0, 2, 4, 5, 5, 7], np.int64)
    good = np.array([0, 3, 4, 7, 8], np.int64)        # tiles of 2 code positions
    r = O.decode_with_sidecar("fsst8", codes, off, db, dl, good, 2)
    assert r.status == O.OK and bytes(r.out_bytes) == b"abcxabcc" and list(r.out_off) == [0, 3, 4, 6, 6, 8]
    for bad in ([0, 3, 4, 7, 9], [1, 3, 4, 7, 8], [0, 4, 4, 7, 8], [0, -3, 4, 7, 8], [0, 3, 4, 7, 1 << 62]):
        assert O.decode_with_sidecar("fsst8", codes, off, db, dl, np.array(bad, np.int64), 2).status == O.ESIDECAR
    # a wrong sidecar and too little room: ESIDECAR; the right one: ECAPACITY
    assert O.decode_with_sidecar("fsst8", codes, off, db, dl, np.array([0, 3, 5, 7, 8]), 2,
                                 out_capacity=3).status == O.ESIDECAR
    assert O.decode_with_sidecar("fsst8", codes, off, db, dl, good, 2, out_capacity=3).status == O.ECAPACITY
    # an error in the data wins over a wrong sidecar
    bad_codes = codes.copy()
    bad_codes[5] = 9
    assert O.decode_with_sidecar("fsst8", bad_codes, off, db, dl, good, 2).status == O.EBADCODE
    assert O.sidecar("fsst8", bad_codes, off, db, dl, 2)[0] == O.EBADCODE
    with pytest.raises(ValueError):              # a sidecar of another tiling
        O.decode_with_sidecar("fsst8", codes, off, db, dl, good, 3)


# --------------------------------------------------------------------------- #
# selective decode (take)
# --------------------------------------------------------------------------- #


def source_take(text, text_off, rows):
    """The selected source strings (the generator's text, no decode)."""
    parts = [bytes(text[int(text_off[r]):int(text_off[r + 1])]) for r in rows]
    off = np.concatenate([[0], np.cumsum([len(p) for p in parts])]).astype(np.int64)
    return off, b"".join(parts)


def test_take_by_hand(oracle_mod):
    """Hand-derived: FSST-8 table {0: "ab", 1: "c"}; strings "abc", "x"
    (escape + literal), "ab", "" and "cc"."""
    O = oracle_mod
    db, dl = pack([b"ab", b"c"])
    codes = np.array([0, 1, 255, ord("x"), 0, 1, 1], np.uint8)
    off = np.array([0, 2, 4, 5, 5, 7], np.int64)
    for rows, exp_off, exp in (([4, 0], [0, 2, 5], b"ccabc"), ([1, 1, 3], [0, 1, 2, 2], b"xx"), ([], [0], b""),
                               ([3], [0, 0], b""), ([2, 1, 0], [0, 2, 3, 6], b"abxabc")):
        r = O.take("fsst8", codes, off, db, dl, rows)
        assert r.status == O.OK and list(r.out_off) == exp_off and bytes(r.out_bytes) == exp, rows


@pytest.mark.parametrize("order", ["sorted", "random", "repeats", "all", "reversed"])
def test_take_is_the_source_strings(oracle_mod, datagen_mod, order):
    """Against the generator's own strings, for three codecs."""
    rng = np.random.default_rng(len(order))
    cols = [(datagen_mod.fsst_small(), None),
            (datagen_mod.onpair_urls(target_bytes=1 << 20, sample_bytes=1 << 20), None)]
    c12 = datagen_mod.onpair12_urls(target_bytes=1 << 19)
    cols.append((c12, c12.stats["n_codes"]))
    for c, n_codes in cols:
        n = c.n_strings
        if order == "sorted":
            rows = np.sort(rng.choice(n, n // 10, replace=False))
        elif order == "random":
            rows = rng.choice(n, n // 10, replace=False)
        elif order == "repeats":
            rows = rng.integers(0, n, n // 5)
        elif order == "all":
            rows = np.arange(n)
        else:
            rows = np.arange(n)[::-1]
        r = oracle_mod.take(c.codec, c.codes, c.code_off, c.dict_bytes, c.dict_lens, rows, n_codes=n_codes)
        exp_off, exp = source_take(c.text, c.text_off, rows)
        assert r.status == 0 and np.array_equal(r.out_off, exp_off) and bytes(r.out_bytes) == exp, c.codec


def test_take_errors(oracle_mod):
    O = oracle_mod
    db, dl = pack([b"ab", b"c"])
    codes = np.array([0, 1, 255, ord("x"), 0, 9, 1], np.uint8)      # string 3 ("9") has a bad code
    off = np.array([0, 2, 4, 5, 6, 7], np.int64)
    assert O.take("fsst8", codes, off, db, dl, [0, 5]).status == O.EOFFSETS
    assert O.take("fsst8", codes, off, db, dl, [-1]).status == O.EOFFSETS
    assert O.take("fsst8", codes, off, db, dl, [0, 1]).status == O.OK          # the bad string is not selected
    assert O.take("fsst8", codes, off, db, dl, [0, 3]).status == O.EBADCODE
    # a budget of codes: 2 + 2 codes selected
    assert O.take("fsst8", codes, off, db, dl, [0, 1], max_codes=3).status == O.ENOMEM
    assert O.take("fsst8", codes, off, db, dl, [0, 1], max_codes=4).status == O.OK
    # EOFFSETS before ENOMEM before data errors
    assert O.take("fsst8", codes, off, db, dl, [3, 7], max_codes=0).status == O.EOFFSETS
    assert O.take("fsst8", codes, off, db, dl, [3], max_codes=0).status == O.ENOMEM
    # offsets of a selected string out of order; those of others are not read
    off2 = np.array([0, 2, 1, 5, 6, 7], np.int64)
    assert O.take("fsst8", codes, off2, db, dl, [1]).status == O.EOFFSETS
    assert O.take("fsst8", codes, off2, db, dl, [3, 4]).status == O.EBADCODE
    # capacity
    r = O.take("fsst8", codes, off, db, dl, [0, 2], out_capacity=2)
    assert r.status == O.ECAPACITY and list(r.out_off) == [0, 3, 5]


# --------------------------------------------------------------------------- #
# errors and precedence
# --------------------------------------------------------------------------- #


def test_errors_and_precedence(oracle_mod):
    O = oracle_mod
    db, dl = pack([b"ab", b"c"])
    u8 = lambda *x: np.array(x, np.uint8)
    i64 = lambda *x: np.array(x, np.int64)
    # offsets
    assert O.decode("fsst8", u8(0, 1), i64(1, 0), db, dl).status == O.EOFFSETS
    assert O.decode("fsst8", u8(0, 1), i64(-1, 2), db, dl).status == O.EOFFSETS
    assert O.decode("fsst8", u8(0, 1), i64(0, 3), db, dl).status == O.EOFFSETS
    # dictionary
    assert O.decode("fsst8", u8(0), i64(0, 1), *pack([b"", b"c"])).status == O.EBADDICT
    assert O.decode("fsst8", u8(0), i64(0, 1), *pack([b"123456789"])).status == O.EBADDICT
    assert O.decode("onpair16", np.array([0], np.uint16), i64(0, 1), *pack([b"x" * 17])).status == O.EBADDICT
    # EBADDICT before EOFFSETS, EOFFSETS before data errors
    assert O.decode("fsst8", u8(9), i64(1, 0), *pack([b""])).status == O.EBADDICT
    assert O.decode("fsst8", u8(9), i64(0, 2), db, dl).status == O.EOFFSETS
    # data errors in stream order
    r = O.decode("fsst8", u8(0, 255, 9), i64(0, 2, 3), db, dl)
    assert r.status == O.EESCAPE and r.err_pos == 1
    r = O.decode("fsst8", u8(9, 255), i64(0, 1, 2), db, dl)
    assert r.status == O.EBADCODE and r.err_pos == 0
    r = O.decode("onpair16", np.array([0, 1, 2], np.uint16), i64(0, 3), db, dl)
    assert r.status == O.EBADCODE and r.err_pos == 2
    # capacity: offsets complete, bytes up to the capacity
    r = O.decode("fsst8", u8(0, 1, 0), i64(0, 2, 3), db, dl, out_capacity=4)
    assert r.status == O.ECAPACITY and list(r.out_off) == [0, 3, 5] and bytes(r.out_bytes) == b"abca"
    r = O.decode("fsst8", u8(0, 1, 0), i64(0, 2, 3), db, dl, out_capacity=5)
    assert r.status == O.OK and bytes(r.out_bytes) == b"abcab"
    # data error before capacity
    assert O.decode("fsst8", u8(0, 1, 7), i64(0, 2, 3), db, dl, out_capacity=1).status == O.EBADCODE
    # argument errors
    assert O.decode("fsst8", u8(0), i64(0, 1), db, dl, index_bits=16).status == O.EINVAL


@pytest.mark.slow
def test_overflow_int32_boundary(oracle_mod):
    """32-bit offsets hold a total of exactly INT32_MAX but not INT32_MAX + 1
    (capacity 0 so that no output is written: the status is then ECAPACITY
    when the offsets fit)."""
    db, dl = pack([b"0123456789abcdef", b"0123456789abcde"])
    n = 2 ** 27                              # n tokens of 16 bytes = 2**31 bytes
    codes = np.zeros(n, np.uint16)
    r = oracle_mod.decode("onpair16", codes, np.array([0, n], np.int32), db, dl, out_capacity=0)
    assert r.status == oracle_mod.EOVERFLOW and r.total == 2 ** 31
    codes[-1] = 1                            # total = 2**31 - 1 = INT32_MAX
    r = oracle_mod.decode("onpair16", codes, np.array([0, n], np.int32), db, dl, out_capacity=0)
    assert r.status == oracle_mod.ECAPACITY and r.total == 2 ** 31 - 1
    r = oracle_mod.decode("onpair16", codes, np.array([0, n], np.int64), db, dl, out_capacity=2 ** 31 - 1)
    assert r.status == oracle_mod.OK
