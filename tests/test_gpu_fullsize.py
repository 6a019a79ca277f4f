"""Parity at the full workload sizes, in the launch configuration the
benchmark times (automatic tiling, resident grid, asynchronous status):

- the 1 GiB FSST-8 log column (with the n-gram table and with the trained
  table), the 1 GiB OnPair-16 URL column and their 12-bit packed counterparts
  (OnPair-12 URLs, FSST-12 logs), in both ways to the tile positions (three
  phases, which the benchmark times, and the single pass): the whole
  output must equal the generator's source text and offsets (decoding is
  lossless, so that is the expected result at any size), and sampled runs of
  strings across the column are checked against the oracle one run at a time;
- the 256-column batch (2.26 GB) as one replayed graph: every column equals its
  source text, and sampled runs of each of a few columns match the oracle;
- the 1 GiB FSST-8 and OnPair-16 columns through the stored-sidecar decode and
  a 10% selection in random order, against the source offsets and text."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_15034_amd as fd
    fd.lib()
    yield


def sample_runs(n_strings, rng, n_runs=40, run=50):
    """Runs of consecutive strings: the first, the last and random ones."""
    starts = [0, max(0, n_strings - run)] + list(rng.integers(0, max(1, n_strings - run), size=n_runs))
    return [(int(a), int(min(n_strings, a + run))) for a in starts]


def check_runs_against_oracle(col, out_off, out, rng, n_runs=40):
    import oracle
    co = col.code_off.astype(np.int64)
    codec, codes = col.codec, col.codes
    if codec == "onpair12":          # runs of a packed stream: the oracle's unpacked codes
        codec, codes = "onpair16", oracle.unpack12_np(col.codes, int(col.stats["n_codes"]))
    for a, b in sample_runs(col.n_strings, rng, n_runs):
        c0, c1 = int(co[a]), int(co[b])
        exp = oracle.decode(codec, codes[c0:c1], co[a:b + 1] - c0, col.dict_bytes, col.dict_lens)
        assert exp.status == 0
        rel = out_off[a:b + 1] - out_off[a]
        assert np.array_equal(rel, exp.out_off), (col.name, a, b)
        assert np.array_equal(out[int(out_off[a]):int(out_off[b])], exp.out_bytes), (col.name, a, b)


@pytest.mark.parametrize("workload,seed", [("fsst_logs_ngram", 2), ("fsst_logs", 2), ("onpair_urls", 3),
                                           ("onpair12_urls", 6), ("fsst12_logs", 7)])
def test_full_column(datagen_mod, oracle_mod, workload, seed):
    import torch
    import paper_2609_15034_amd as fd
    col = getattr(datagen_mod, workload)(seed=seed)
    print(f"{workload}: {col.stats}", flush=True)
    dev = torch.device("cuda")
    codes = torch.from_numpy(col.codes.view(np.int16) if col.codec == "onpair16" else col.codes).to(dev)
    code_off = torch.from_numpy(col.code_off).to(dev)
    d = fd.Dict(col.codec, torch.from_numpy(col.dict_bytes).to(dev), torch.from_numpy(col.dict_lens).to(dev))
    guard = 4096
    buf = torch.full((col.decoded_bytes + guard,), 0xA5, dtype=torch.uint8, device=dev)
    out = buf[:col.decoded_bytes]
    out_off = torch.full((col.n_strings + 1,), -7, dtype=code_off.dtype, device=dev)
    ws = fd.alloc_workspace(col.codec, fd.codes_in(col.codec, codes), col.n_strings)
    status = torch.full((1,), -1, dtype=torch.int32, device=dev)
    text = torch.from_numpy(col.text).to(dev)
    text_off = torch.from_numpy(col.text_off).to(dev)
    for mode in (0, 1):
        tu = {"mode": mode, "tile_codes": 0, "grid": 0, "reserved": 0}
        out.fill_(0x5A)
        out_off.fill_(-7)
        for _ in range(2):    # twice: the second run reuses the workspace as the benchmark does
            assert fd.decode_into(d, codes, code_off, out_off, out, ws, status=status, async_=True,
                                  tuning=tu) == fd.OK
            torch.cuda.synchronize()
            assert int(status.item()) == fd.OK, mode
        assert torch.equal(out, text), mode
        assert torch.equal(out_off.to(torch.int64), text_off), mode
        assert bool((buf[col.decoded_bytes:] == 0xA5).all()), "write past the output"
    rng = np.random.default_rng(seed + 100)
    check_runs_against_oracle(col, out_off.cpu().numpy().astype(np.int64), out.cpu().numpy(), rng)


def test_full_batch(datagen_mod, oracle_mod):
    import torch
    import paper_2609_15034_amd as fd
    cols = datagen_mod.batch_columns(seed=4)
    dev = torch.device("cuda")
    tups, bufs = [], []
    for c in cols:
        codes = torch.from_numpy(c.codes if c.codec == "fsst8" else c.codes.view(np.int16)).to(dev)
        code_off = torch.from_numpy(c.code_off).to(dev)
        d = fd.Dict(c.codec, torch.from_numpy(c.dict_bytes).to(dev), torch.from_numpy(c.dict_lens).to(dev))
        buf = torch.full((c.decoded_bytes + 64,), 0xA5, dtype=torch.uint8, device=dev)
        bufs.append(buf)
        tups.append((d, codes, code_off, torch.full((c.n_strings + 1,), -7, dtype=code_off.dtype, device=dev),
                     buf[:c.decoded_bytes]))
    ws = torch.empty(fd.batch_workspace_size(tups, None), dtype=torch.uint8, device=dev)
    status = torch.full((len(tups) + 1,), -1, dtype=torch.int32, device=dev)
    for _ in range(3):        # autotune on the first call, then graph replays
        assert fd.batch_decode(tups, ws, status=status, async_=True, graph=True) == fd.OK
        torch.cuda.synchronize()
        assert int(status[-1].item()) == fd.OK
    assert bool((status == 0).all())
    for c, t, buf in zip(cols, tups, bufs):
        assert torch.equal(t[4], torch.from_numpy(c.text).to(dev)), c.name
        assert torch.equal(t[3].to(torch.int64), torch.from_numpy(c.text_off).to(dev)), c.name
        assert bool((buf[c.decoded_bytes:] == 0xA5).all()), c.name
    rng = np.random.default_rng(41)
    for k in rng.choice(len(cols), size=6, replace=False):
        c, t = cols[int(k)], tups[int(k)]
        check_runs_against_oracle(c, t[3].cpu().numpy().astype(np.int64), t[4].cpu().numpy(), rng, n_runs=8)


@pytest.mark.parametrize("workload,seed", [("fsst_logs", 2), ("onpair_urls", 3)])
def test_full_column_sidecar_and_take(datagen_mod, workload, seed):
    """The 1 GiB columns through the stored-sidecar decode and a 10% selection
    in random order, as the benchmark runs them: the sidecar equals the
    output position of every tile's first code (the source offsets of the
    string holding it plus the oracle's walk of that string), both outputs
    equal the source text."""
    import torch
    import paper_2609_15034_amd as fd
    col = getattr(datagen_mod, workload)(seed=seed)
    dev = torch.device("cuda")
    codes = torch.from_numpy(col.codes.view(np.int16) if col.codec == "onpair16" else col.codes).to(dev)
    code_off = torch.from_numpy(col.code_off).to(dev)
    d = fd.Dict(col.codec, torch.from_numpy(col.dict_bytes).to(dev), torch.from_numpy(col.dict_lens).to(dev))
    text = torch.from_numpy(col.text).to(dev)
    to = np.asarray(col.text_off, np.int64)
    # sidecar: built on the device, checked against the source offsets, then decoded with
    import oracle
    T, n_entries = fd.sidecar_layout(col.codec, codes.numel(), col.n_strings)
    sc = fd.sidecar_build(d, codes, code_off)
    # every tile start's output position: the source strings' offsets plus
    # the oracle's walk of the string holding the tile start
    st, exp = oracle.sidecar(col.codec, col.codes, col.code_off, col.dict_bytes, col.dict_lens, T,
                             string_offsets=to)
    assert st == 0 and len(exp) == n_entries
    assert np.array_equal(sc.cpu().numpy(), exp)
    out = torch.full((col.decoded_bytes + 64,), 0xA5, dtype=torch.uint8, device=dev)
    out_off = torch.full((col.n_strings + 1,), -7, dtype=code_off.dtype, device=dev)
    ws = fd.alloc_workspace(col.codec, codes.numel(), col.n_strings)
    st = fd.decode_sidecar_into(d, codes, code_off, sc, out_off, out[:col.decoded_bytes], ws)
    assert st == fd.OK
    assert torch.equal(out[:col.decoded_bytes], text)
    assert torch.equal(out_off.to(torch.int64), torch.from_numpy(to).to(dev))
    assert bool((out[col.decoded_bytes:] == 0xA5).all())
    del out, out_off, ws, sc
    # take: 10% of the rows in random order
    rng = np.random.default_rng(seed + 200)
    rows = rng.choice(col.n_strings, col.n_strings // 10, replace=False)
    lens = to[rows + 1] - to[rows]
    D = int(lens.sum())
    ws = torch.empty(fd.take_workspace_size(col.codec, codes.numel(), col.n_strings, len(rows), codes.numel()),
                     dtype=torch.uint8, device=dev)
    out = torch.full((D + 64,), 0xA5, dtype=torch.uint8, device=dev)
    out_off = torch.full((len(rows) + 1,), -7, dtype=code_off.dtype, device=dev)
    st = fd.decode_take_into(d, codes, code_off, torch.from_numpy(rows.astype(np.int64)).to(dev), codes.numel(),
                             out_off, out[:D], ws)
    assert st == fd.OK
    exp_off = np.concatenate([[0], np.cumsum(lens)])
    assert np.array_equal(out_off.cpu().numpy().astype(np.int64), exp_off)
    lens_t = torch.from_numpy(lens).to(dev)
    idx = torch.repeat_interleave(torch.from_numpy(to[rows]).to(dev) - torch.from_numpy(exp_off[:-1]).to(dev),
                                  lens_t) + torch.arange(D, device=dev)
    assert torch.equal(out[:D], text[idx])
    assert bool((out[D:] == 0xA5).all())
