"""GPU parity for selective decode (fd_decode_take): the strings a row list
names, decoded through the C ABI, against the CPU oracle's take, bit-exact in
status, Arrow offsets and bytes; selections in every order, with repeats,
empty and whole; errors in selected and unselected strings; the code budget."""
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


def selected_codes(c, rows):
    co = np.asarray(c.code_off, np.int64)
    rows = np.asarray(rows, np.int64)
    return int((co[rows + 1] - co[rows]).sum()) if len(rows) else 0


def gpu_take(c, rows, *, max_codes=None, tuning=None, cap=None, async_=False, misalign=0):
    """fd_decode_take on the GPU: (status, out_off, out_bytes), guards checked."""
    import torch
    import paper_2609_15034_amd as fd
    n_codes = n_codes_of(c)
    raw = np.ascontiguousarray(c.codes)
    if misalign:
        b = np.frombuffer(raw.tobytes(), np.uint8)
        buf = torch.zeros(len(b) + misalign + 16, dtype=torch.uint8, device="cuda")
        buf[misalign:misalign + len(b)] = torch.from_numpy(b.copy()).cuda()
        codes = buf[misalign:misalign + len(b)]
    else:
        codes = torch.from_numpy((raw.view(np.int16) if c.codec == "onpair16" else raw).copy()).cuda()
    off = torch.from_numpy(np.ascontiguousarray(c.code_off)).cuda()
    d = fd.Dict(c.codec, torch.from_numpy(np.ascontiguousarray(c.dict_bytes, np.uint8)).cuda(),
                torch.from_numpy(np.ascontiguousarray(c.dict_lens, np.uint8)).cuda())
    rows_t = torch.from_numpy(np.ascontiguousarray(rows, np.int64)).cuda()
    if max_codes is None:
        max_codes = selected_codes(c, rows) if len(rows) and min(rows) >= 0 and max(rows) < c.n_strings else n_codes
    if cap is None:
        cap = max(1, max_codes) * (8 if c.codec == "fsst8" else 16)
    g = GuardedOut(cap, len(rows) + 1, off.dtype)
    ws = torch.empty(fd.take_workspace_size(c.codec, n_codes, c.n_strings, len(rows), max_codes, tuning),
                     dtype=torch.uint8, device="cuda")
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda") if async_ else None
    st = fd.decode_take_into(d, codes, off, rows_t, max_codes, g.off, g.out, ws, status=status, async_=async_,
                             tuning=tuning, n_codes=n_codes)
    torch.cuda.synchronize()
    if async_:
        assert st == fd.OK
        st = int(status.item())
    g.check_guards()
    return st, g.off.cpu().numpy().astype(np.int64), g.out.cpu().numpy()


def assert_take(c, rows, **kw):
    import oracle
    extra = {"n_codes": n_codes_of(c)} if c.codec == "onpair12" else {}
    mc = kw.get("max_codes")
    exp = oracle.take(c.codec, c.codes, c.code_off, c.dict_bytes, c.dict_lens, rows, max_codes=mc,
                      out_capacity=kw.get("cap"), **extra)
    st, off, out = gpu_take(c, rows, **kw)
    assert st == exp.status, (st, exp.status)
    if exp.status in (0, 4):
        assert np.array_equal(off, exp.out_off)
        assert np.array_equal(out[:len(exp.out_bytes)], exp.out_bytes)
    return exp


@pytest.fixture(scope="module")
def cols(datagen_mod):
    return {"fsst_small": datagen_mod.fsst_small(),
            "fsst_logs": datagen_mod.fsst_logs(target_bytes=8 << 20),
            "onpair_urls": datagen_mod.onpair_urls(target_bytes=8 << 20, sample_bytes=2 << 20),
            "onpair12_urls": datagen_mod.onpair12_urls(target_bytes=8 << 20),
            "fsst12_logs": datagen_mod.fsst12_logs(target_bytes=4 << 20)}


def make_rows(n, order, rng):
    if order == "sorted10":
        return np.sort(rng.choice(n, max(1, n // 10), replace=False))
    if order == "random10":
        return rng.choice(n, max(1, n // 10), replace=False)
    if order == "repeats":
        return rng.integers(0, n, max(1, n // 3))
    if order == "all":
        return np.arange(n)
    if order == "reversed":
        return np.arange(n)[::-1].copy()
    if order == "ends":
        return np.array([n - 1, 0, n - 1, 0])
    if order == "one":
        return np.array([n // 2])
    return np.zeros(0, np.int64)


@pytest.mark.parametrize("name", ["fsst_small", "fsst_logs", "onpair_urls", "onpair12_urls", "fsst12_logs"])
@pytest.mark.parametrize("order", ["sorted10", "random10", "repeats", "all", "reversed", "ends", "one", "none"])
def test_take(cols, name, order):
    c = cols[name]
    rows = make_rows(c.n_strings, order, np.random.default_rng(len(order) + len(name)))
    exp = assert_take(c, rows)
    assert exp.status == 0
    co = np.asarray(c.text_off, np.int64)
    if len(rows):                                  # the generator's own strings
        assert exp.out_off[-1] == int((co[rows + 1] - co[rows]).sum())


@pytest.mark.parametrize("tuning", [{"mode": 0, "tile_codes": 16, "grid": 0, "reserved": 0},
                                    {"mode": 0, "tile_codes": 400, "grid": 3, "reserved": 0},
                                    {"mode": 0, "tile_codes": 0, "grid": 0, "reserved": 0},
                                    {"mode": 1, "tile_codes": 16, "grid": 0, "reserved": 0},
                                    {"mode": 1, "tile_codes": 400, "grid": 3, "reserved": 0},
                                    {"mode": 1, "tile_codes": 0, "grid": 0, "reserved": 0}])
@pytest.mark.parametrize("name", ["fsst_logs", "onpair12_urls"])
def test_take_tuning(cols, name, tuning):
    c = cols[name]
    rows = make_rows(c.n_strings, "random10", np.random.default_rng(8))
    assert assert_take(c, rows, tuning=tuning).status == 0


@pytest.mark.parametrize("misalign", [1, 3])
def test_take_unaligned_12bit(cols, misalign):
    c = cols["onpair12_urls"]
    rows = make_rows(c.n_strings, "repeats", np.random.default_rng(misalign))
    assert assert_take(c, rows, misalign=misalign).status == 0


@pytest.mark.parametrize("name", ["fsst_logs", "onpair_urls", "onpair12_urls"])
@pytest.mark.parametrize("order", ["sorted10", "random10", "repeats", "all", "ends", "one", "none"])
def test_take_three_phases(cols, name, order):
    """The selection decoded by the three phases (their expand pass takes
    tiles from the split queues), at the default and at small tiles."""
    c = cols[name]
    rows = make_rows(c.n_strings, order, np.random.default_rng(len(order) + 3 * len(name)))
    for tc in (0, 64):
        tuning = {"mode": 1, "tile_codes": tc, "grid": 0, "reserved": 0}
        assert assert_take(c, rows, tuning=tuning).status == 0


@pytest.mark.parametrize("mode", [0, 1])
def test_take_errors(cols, mode):
    c = cols["fsst_logs"]
    n = c.n_strings
    tu = {"mode": mode, "tile_codes": 0, "grid": 0, "reserved": 0}
    rng = np.random.default_rng(4)
    rows = make_rows(n, "random10", rng)
    # rows outside the column
    for bad in (n, -1, 1 << 40):
        r2 = rows.copy()
        r2[len(r2) // 2] = bad
        assert assert_take(c, r2, max_codes=n_codes_of(c), tuning=tu).status == 3 + 4     # EOFFSETS
    # a code budget one short, and exactly enough
    need = selected_codes(c, rows)
    assert assert_take(c, rows, max_codes=need - 1, tuning=tu).status == 9                 # ENOMEM
    assert assert_take(c, rows, max_codes=need, tuning=tu).status == 0
    # capacity, async
    total = int(assert_take(c, rows, tuning=tu).out_off[-1])
    assert assert_take(c, rows, cap=total - 1, tuning=tu).status == 4
    assert assert_take(c, rows, async_=True, tuning=tu).status == 0


def test_take_errors_in_strings(datagen_mod):
    """A bad code in a selected string is reported; one in an unselected string
    is not seen."""
    c = datagen_mod.random_onpair(seed=9, n_codes=1 << 16, n_strings=1000, n_tok=1000)
    co = np.asarray(c.code_off, np.int64)
    bad_row = next(j for j in range(500, 1000) if co[j + 1] > co[j])      # a non-empty string
    codes = c.codes.copy()
    codes[co[bad_row]] = 1000                   # not a token of the 1,000-token dictionary
    c2 = type(c)(**{**c.__dict__, "codes": codes})
    rows_with = np.array([3, bad_row, 7]) if bad_row not in (3, 7) else np.array([bad_row])
    rows_without = np.array([r for r in range(0, 1000, 7) if r != bad_row])
    for mode in (0, 1):
        tu = {"mode": mode, "tile_codes": 0, "grid": 0, "reserved": 0}
        assert assert_take(c2, rows_with, tuning=tu).status == 2
        assert assert_take(c2, rows_without, tuning=tu).status == 0


def test_take_automatic_mode_large_selection(datagen_mod):
    """Without a tuning a selection expected to span at least four times as
    many tiles as resident workgroups runs the three phases (the profiler sees
    its totals launch): every row of a 96 MiB log column, in order and
    reversed."""
    import paper_2609_15034_amd as fd
    c = datagen_mod.fsst_logs(seed=43, target_bytes=96 << 20)
    for rows in (np.arange(c.n_strings), np.arange(c.n_strings)[::-1].copy()):
        fd.profile_begin(("totals", "decode"), 64)
        assert assert_take(c, rows).status == 0
        assert "totals" in fd.profile_end()
