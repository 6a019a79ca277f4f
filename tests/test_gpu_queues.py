"""GPU parity of the tile queues: a decode that needs no order (the expand
pass of the three phases, the sidecar decode) takes its tiles from eight
contiguous ranges, each with its own counter, every workgroup starting on
range blockIdx % 8 and moving on when its range is used up.  These cases put
the tile count on both sides of the range count (ranges that are empty, one
tile each, uneven), with grids smaller than the range count (one workgroup
walks all eight) and not dividing it, and reuse one workspace for decodes of
different sizes (the counters start from zero on every call).  The oracle
decides every byte and offset."""
import numpy as np
import pytest

from gpu_util import assert_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_15034_amd as fd
    fd.lib()   # raises when the library is not built
    yield


def tu(mode, tc, grid):
    return {"mode": mode, "tile_codes": tc, "grid": grid, "reserved": 0}


def tile_codes_for_count(n_codes, k, quantum):
    """The tile size (a multiple of `quantum`) that gives about k tiles."""
    return max(quantum, -(-(-(-n_codes // k)) // quantum) * quantum)


@pytest.mark.parametrize("k", [1, 2, 7, 8, 9, 17, 100])
@pytest.mark.parametrize("grid", [0, 1, 3, 9])
def test_fsst_tile_counts_around_the_queue_count(datagen_mod, k, grid):
    c = datagen_mod.fsst_small(seed=31, n_strings=min(3000, 150 * k))
    T = tile_codes_for_count(len(c.codes), k, 16)
    assert T <= 8176
    assert_parity("fsst8", c.codes, c.code_off, c.dict_bytes, c.dict_lens, tuning=tu(1, T, grid))


@pytest.mark.parametrize("k", [3, 8, 11, 64])
@pytest.mark.parametrize("grid", [1, 5])
def test_onpair_tile_counts_around_the_queue_count(datagen_mod, k, grid):
    c = datagen_mod.onpair_urls(seed=32, target_bytes=min(256 << 10, (20 << 10) * k), sample_bytes=256 << 10)
    T = tile_codes_for_count(len(c.codes), k, 8)
    assert T <= 4088
    assert_parity("onpair16", c.codes, c.code_off, c.dict_bytes, c.dict_lens, tuning=tu(1, T, grid))


def test_workspace_reused_across_sizes(datagen_mod):
    """One workspace, three decodes in a row (large, small, large): each
    matches the oracle, so no queue counter carries over between calls."""
    import torch
    import oracle
    import paper_2609_15034_amd as fd
    cols = [datagen_mod.fsst_logs(seed=33, target_bytes=2 << 20),
            datagen_mod.fsst_small(seed=34, n_strings=500),
            datagen_mod.fsst_logs(seed=35, target_bytes=3 << 20)]
    tuning = tu(1, 256, 0)
    big = max(cols, key=lambda c: len(c.codes))
    ws = fd.alloc_workspace("fsst8", len(big.codes), max(len(c.code_off) - 1 for c in cols), tuning)
    for c in cols:
        exp = oracle.decode("fsst8", c.codes, c.code_off, c.dict_bytes, c.dict_lens)
        assert exp.status == 0
        d = fd.Dict("fsst8", torch.from_numpy(c.dict_bytes).cuda(), torch.from_numpy(c.dict_lens).cuda())
        codes = torch.from_numpy(c.codes).cuda()
        off = torch.from_numpy(np.ascontiguousarray(c.code_off)).cuda()
        out = torch.empty(len(exp.out_bytes), dtype=torch.uint8, device="cuda")
        oo = torch.empty(len(c.code_off), dtype=off.dtype, device="cuda")
        st = fd.decode_into(d, codes, off, oo, out, ws, tuning=tuning)
        assert st == fd.OK
        assert np.array_equal(oo.cpu().numpy().astype(np.int64), exp.out_off)
        assert np.array_equal(out.cpu().numpy(), exp.out_bytes)
