#!/usr/bin/env python3
"""Decode throughput of one MI355X on a synthetic string column.

A step is one full decode of the column (the whole hot path: workspace reset,
code load, escape parity, decoded-length scan, tile cursors, LDS assembly,
16-byte drain, Arrow offsets) with every input resident in HBM and the
dictionary prepared beforehand (the paper repacks dictionaries before timing).
The tile cursors come from the three-phase path by default (--mode 1: tile
totals streamed, scanned, then the expand pass), the fastest way on these
columns; --mode 0 takes the single pass with its decoupled look-back.
Default workload: FSST-8 log lines, 1 GiB decoded, int64 offsets, with the table
built as the configuration states it (top-255 frequent 1-8 byte n-grams of a
1 MiB sample); "fsst_logs" is the same text with an FSST-style trained table.

Prints one JSON line:
  value        decoded GB/s (1e9 output bytes per second) = decoded bytes /
               mean step time
  roofline     the dominant kernel (k_decode): algorithmic bytes (decoded bytes
               + code bytes + code offsets read + Arrow offsets written +
               dictionary) / its mean launch duration, timed inside the timed
               steps with HIP events the library records on its launch stream,
               against the 8 TB/s HBM peak; "step" holds the same over the whole
               step, "kernels_us" every kernel's mean duration; `traffic` is the
               HBM bytes per launch from the committed rocprofv3 counter summary
               when it was taken on the current kernel source, else null
  cpu_baseline the CPU oracle on this host's cores over the same column
  bit_exact    GPU output == the generated source text (bytes and offsets)

  python bench.py [--workload fsst_logs_ngram|fsst_logs|onpair_urls|onpair12_urls|fsst12_logs|fsst_small|
                              batch256|serve]
                  [--steps K] [--warmup W] [--sidecar]

--sidecar times the decode with output positions read from a stored sidecar
(built once before timing) instead of the look-back.

The default run (fsst_logs) also reports the other 1 GiB columns' rates, the
sidecar decode against the look-back on the FSST-8 and OnPair-16 columns
("sidecar"), selective decode of row subsets of those columns ("take"), and,
in "batch" and "serve", short runs of the batched workload
(256 columns in one replayed HIP graph, against the same columns decoded one
call each) and of the served workload (5,000 Poisson arrivals per load into
the continuous-batching server at 0.5, 0.7, 0.9 and 1.5 x its batch capacity,
p50/p99 latency); --no-extra skips them.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "decoded GB/s per GPU (fraction of HBM peak), bit-exact; p50/p99 latency served"
WORKLOADS = {
    "fsst_logs_ngram": dict(codec="fsst8", desc="FSST-8 log lines, 1 GiB decoded, int64 offsets; table = top-255 "
                                                "frequent 1-8 byte n-grams of a 1 MiB sample, greedy longest match",
                            table="top-255 1-8-byte n-grams of a 1 MiB sample (count x length)"),
    "fsst_logs": dict(codec="fsst8", desc="FSST-8 log lines, 1 GiB decoded, int64 offsets; table trained by "
                                          "FSST-style rounds on a 1 MiB sample",
                      table="FSST-style trained rounds on a 1 MiB sample"),
    "onpair_urls": dict(codec="onpair16", desc="OnPair-16 URL/identifier strings, 1 GiB decoded, int64 offsets"),
    "onpair12_urls": dict(codec="onpair12", desc="OnPair-12 (12-bit packed codes, 4,096 tokens) URL/identifier "
                                                 "strings, 1 GiB decoded, int64 offsets"),
    "fsst12_logs": dict(codec="onpair12", desc="FSST-12 (12-bit packed codes, 4,096 symbols of 1-8 bytes, no "
                                               "escapes) log lines, 1 GiB decoded, int64 offsets"),
    "fsst_small": dict(codec="fsst8", desc="FSST-8 printable strings, 10,000 strings, int32 offsets"),
    "batch256": dict(codec="mixed", desc="256 columns, decoded sizes log-uniform 4 KB-64 MB, FSST-8 / OnPair-16 "
                                        "50/50, a dictionary per column, one replayed HIP graph"),
    "serve": dict(codec="mixed", desc="Poisson arrivals of chunks log-uniform 64 KB-32 MB, 32 device-resident "
                                     "dictionaries, 16 GB in flight, continuous batching"),
}
KERNEL_SOURCES = ["paper_2609_15034_amd/csrc/fd_kernels.hip", "paper_2609_15034_amd/csrc/fd_internal.h",
                  "paper_2609_15034_amd/csrc/fd_host.cpp"]


def positions_label(mode: int, sidecar: bool) -> str:
    """How the step finds each tile's output position."""
    if sidecar:
        return "stored sidecar"
    return "look-back (single pass)" if mode == 0 else "three phases (tile totals, scan, expand)"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def make_column(name: str, seed: int | None):
    import datagen
    if name == "fsst_logs_ngram":
        return datagen.fsst_logs_ngram(seed=seed or 2)
    if name == "fsst_logs":
        return datagen.fsst_logs(seed=seed or 2)
    if name == "onpair_urls":
        return datagen.onpair_urls(seed=seed or 3)
    if name == "fsst_small":
        return datagen.fsst_small(seed=seed or 1)
    if name == "onpair12_urls":
        return datagen.onpair12_urls(seed=seed or 6)
    if name == "fsst12_logs":
        return datagen.fsst12_logs(seed=seed or 7)
    raise ValueError(name)


def algorithmic_bytes(col) -> int:
    """Bytes the decode must move at minimum: write the decoded bytes, read the
    codes of the decoded range, read the code offsets, write the Arrow offsets,
    read the dictionary once."""
    n_used = int(col.code_off[-1] - col.code_off[0])
    code_bytes = {"fsst8": n_used, "onpair16": 2 * n_used, "onpair12": (12 * n_used + 7) // 8}[col.codec]
    w_off = col.code_off.dtype.itemsize
    return (col.decoded_bytes + code_bytes + 2 * (col.n_strings + 1) * w_off
            + int(col.dict_bytes.size + col.dict_lens.size))


def copy_calibration(nbytes: int, reps: int = 5):
    """A plain device copy of a known size (the reference for the counter
    scaling of FETCH_SIZE / WRITE_SIZE and an achievable-bandwidth ceiling)."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    src.fill_(7)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = 1e30
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b) / 1e3)
    return 2 * nbytes / best / 1e9


def cpu_model() -> str:
    """The host CPU's model name (Linux), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def read_traffic(workload: str, src_hash: str):
    path = os.path.join(ROOT, "profiles", f"decode_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha") != src_hash:
        return None
    return t


def _upload_column(col, dev):
    import numpy as np
    import torch
    codes_np = col.codes.view(np.int16) if col.codec == "onpair16" else col.codes
    return torch.from_numpy(codes_np).to(dev), torch.from_numpy(col.code_off).to(dev)


def _events_time(fn, steps, warmup):
    """Mean seconds per call of fn() over `steps` calls after `warmup`, timed
    with events on the current stream (the stream the library launches on)."""
    import numpy as np
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    evs[0].record()
    for i in range(steps):
        fn()
        evs[i + 1].record()
    torch.cuda.synchronize()
    per = np.array([evs[i].elapsed_time(evs[i + 1]) / 1e3 for i in range(steps)])
    return float(per.mean()), per


def single_rate(workload: str, steps: int = 10, seed: int | None = None, mode: int = 1) -> float:
    """Decoded GB/s of one 1 GiB single-column decode (the c2 / c3 reference
    rates; mode 1: the three-phase path, 0: the single pass)."""
    import numpy as np
    import torch
    import paper_2609_15034_amd as fd
    col = make_column(workload, seed)
    dev = torch.device("cuda")
    codes, code_off = _upload_column(col, dev)
    d = fd.Dict(col.codec, torch.from_numpy(col.dict_bytes).to(dev), torch.from_numpy(col.dict_lens).to(dev))
    out = torch.empty(col.decoded_bytes, dtype=torch.uint8, device=dev)
    out_off = torch.empty(col.n_strings + 1, dtype=code_off.dtype, device=dev)
    tu = {"mode": mode, "tile_codes": 0, "grid": 0, "reserved": 0}
    ws = fd.alloc_workspace(col.codec, fd.codes_in(col.codec, codes), col.n_strings, tu)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    mean_s, _ = _events_time(lambda: fd.decode_into(d, codes, code_off, out_off, out, ws, status=st, async_=True,
                                                    tuning=tu), steps, 2)
    if int(st.item()) != fd.OK or not torch.equal(out, torch.from_numpy(col.text).to(dev)):
        raise fd.DecodeError(int(st.item()), f"{workload} mode {mode}: output differs from the source")
    return col.decoded_bytes / mean_s / 1e9


def small_latency(runs: int = 200, mode: int | None = None, seed: int | None = None) -> dict:
    """The small FSST-8 column (10,000 printable strings, int32 offsets): the
    latency of one whole decode call, timed with events around each call on
    the library's stream, over `runs` calls after a warm-up; the output is
    checked against the source strings.  mode None: the library's automatic
    choice (the single pass at this size), as a caller without a tuning
    gets it."""
    import numpy as np
    import torch
    import paper_2609_15034_amd as fd
    col = make_column("fsst_small", seed)
    dev = torch.device("cuda")
    codes, code_off = _upload_column(col, dev)
    d = fd.Dict(col.codec, torch.from_numpy(col.dict_bytes).to(dev), torch.from_numpy(col.dict_lens).to(dev))
    out = torch.empty(col.decoded_bytes, dtype=torch.uint8, device=dev)
    out_off = torch.empty(col.n_strings + 1, dtype=code_off.dtype, device=dev)
    tu = None if mode is None else {"mode": mode, "tile_codes": 0, "grid": 0, "reserved": 0}
    ws = fd.alloc_workspace(col.codec, fd.codes_in(col.codec, codes), col.n_strings, tu)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    _, per = _events_time(lambda: fd.decode_into(d, codes, code_off, out_off, out, ws, status=st, async_=True,
                                                 tuning=tu), runs, 10)
    ok = int(st.item()) == fd.OK and torch.equal(out, torch.from_numpy(col.text).to(dev)) and \
        torch.equal(out_off.to(torch.int64), torch.from_numpy(col.text_off.astype(np.int64)).to(dev))
    us = per * 1e6
    return {"decoded_bytes": col.decoded_bytes, "n_strings": col.n_strings, "runs": runs,
            "mode": "automatic" if mode is None else mode,
            "latency_us": {"min": round(float(us.min()), 2), "p50": round(float(np.median(us)), 2),
                           "p99": round(float(np.percentile(us, 99)), 2)},
            "GBps_at_p50": round(col.decoded_bytes / float(np.median(per)) / 1e9, 3), "bit_exact": bool(ok)}


def sidecar_rates(workload: str, steps: int = 20, seed: int | None = None) -> dict:
    """One 1 GiB column decoded with its output positions taken from a stored
    sidecar (built once before timing, as the paper stores it with the
    column) and with the positions regenerated by the look-back, timed back to
    back; the sidecar decode's output is checked against the source text."""
    import torch
    import paper_2609_15034_amd as fd
    col = make_column(workload, seed)
    dev = torch.device("cuda")
    codes, code_off = _upload_column(col, dev)
    d = fd.Dict(col.codec, torch.from_numpy(col.dict_bytes).to(dev), torch.from_numpy(col.dict_lens).to(dev))
    out = torch.empty(col.decoded_bytes, dtype=torch.uint8, device=dev)
    out_off = torch.empty(col.n_strings + 1, dtype=code_off.dtype, device=dev)
    ws = fd.alloc_workspace(col.codec, fd.codes_in(col.codec, codes), col.n_strings)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    sc = fd.sidecar_build(d, codes, code_off)
    t_sc, _ = _events_time(lambda: fd.decode_sidecar_into(d, codes, code_off, sc, out_off, out, ws, status=st,
                                                          async_=True), steps, 2)
    ok = int(st.item()) == fd.OK and torch.equal(out, torch.from_numpy(col.text).to(dev)) and \
        torch.equal(out_off.to(torch.int64), torch.from_numpy(col.text_off).to(dev))
    lb = {"mode": 0, "tile_codes": 0, "grid": 0, "reserved": 0}      # the single pass (look-back), explicitly
    t_lb, _ = _events_time(lambda: fd.decode_into(d, codes, code_off, out_off, out, ws, status=st, async_=True,
                                                  tuning=lb), steps, 2)
    D = col.decoded_bytes
    return {"sidecar_GBps": round(D / t_sc / 1e9, 2), "lookback_GBps": round(D / t_lb / 1e9, 2),
            "regeneration_cost": round(t_lb / t_sc - 1.0, 3), "sidecar_bytes": int(sc.numel() * 8),
            "bit_exact": bool(ok)}


def take_rates(workload: str, steps: int = 10, seed: int | None = None,
               shares=(0.001, 0.01, 0.1, 0.5, 1.0)) -> dict:
    """Selective decode of one 1 GiB column: random subsets of the rows (a
    share of them, in row order as a filter gives them, and one share in
    random order as a take gives them), each decoded with fd_decode_take and
    checked against the source strings; against the whole-column decode."""
    import numpy as np
    import torch
    import paper_2609_15034_amd as fd
    col = make_column(workload, seed)
    dev = torch.device("cuda")
    codes, code_off = _upload_column(col, dev)
    d = fd.Dict(col.codec, torch.from_numpy(col.dict_bytes).to(dev), torch.from_numpy(col.dict_lens).to(dev))
    n_codes = fd.codes_in(col.codec, codes)
    co = np.asarray(col.code_off, np.int64)
    to = np.asarray(col.text_off, np.int64)
    text = torch.from_numpy(col.text).to(dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = torch.empty(fd.take_workspace_size(col.codec, n_codes, col.n_strings, col.n_strings, n_codes),
                     dtype=torch.uint8, device=dev)
    rng = np.random.default_rng(17)
    out_all = torch.empty(col.decoded_bytes, dtype=torch.uint8, device=dev)
    res = {}
    for share, order in [(x, "row order") for x in shares] + [(0.1, "random order")]:
        k = max(1, int(round(share * col.n_strings)))
        rows = np.sort(rng.choice(col.n_strings, k, replace=False)) if share < 1.0 else np.arange(col.n_strings)
        if order == "random order":
            rng.shuffle(rows)
        D = int((to[rows + 1] - to[rows]).sum())
        rows_t = torch.from_numpy(rows.astype(np.int64)).to(dev)
        out = out_all[:D]
        out_off = torch.empty(k + 1, dtype=code_off.dtype, device=dev)
        fn = lambda: fd.decode_take_into(d, codes, code_off, rows_t, n_codes, out_off, out, ws, status=st,
                                         async_=True)
        t, _ = _events_time(fn, steps, 2)
        # the source strings, gathered on the device for the check
        lens = torch.from_numpy(to[rows + 1] - to[rows]).to(dev)
        idx = torch.repeat_interleave(torch.from_numpy(to[rows]).to(dev) -
                                      torch.cumsum(lens, 0) + lens, lens) + torch.arange(D, device=dev)
        ok = int(st.item()) == fd.OK and torch.equal(out, text[idx])
        res[f"{share:g} {order}"] = {"rows": k, "decoded_bytes": D, "us": round(t * 1e6, 1),
                                     "GBps": round(D / t / 1e9, 2), "Mrows_per_s": round(k / t / 1e6, 1),
                                     "bit_exact": bool(ok)}
        del idx, lens
    return res


def run_batch(steps: int, warmup: int, seed: int | None, n_cols: int = 256, max_bytes: int = 64 << 20,
              check: bool = True, cpu: bool = True, single_rates: dict | None = None):
    """The batched workload: returns a result dict (see the module docstring)."""
    import numpy as np
    import torch
    import datagen
    import paper_2609_15034_amd as fd
    t0 = time.time()
    cols = datagen.batch_columns(seed=seed or 4, n_cols=n_cols, max_bytes=max_bytes)
    D = sum(c.decoded_bytes for c in cols)
    log(f"[batch] generated {n_cols} columns, {D / 1e9:.3f} GB decoded in {time.time() - t0:.1f}s")
    dev = torch.device("cuda")
    tups, dicts, outs = [], [], []
    for c in cols:
        codes, code_off = _upload_column(c, dev)
        d = fd.Dict(c.codec, torch.from_numpy(c.dict_bytes).to(dev), torch.from_numpy(c.dict_lens).to(dev))
        out = torch.empty(c.decoded_bytes, dtype=torch.uint8, device=dev)
        out_off = torch.empty(c.n_strings + 1, dtype=code_off.dtype, device=dev)
        dicts.append(d)
        outs.append((out, out_off))
        tups.append((d, codes, code_off, out_off, out))
    ws = torch.empty(fd.batch_workspace_size(tups), dtype=torch.uint8, device=dev)
    status = torch.zeros(len(tups) + 1, dtype=torch.int32, device=dev)
    t1 = time.time()
    st = fd.batch_decode(tups, ws, status=status)             # first call: the autotuner picks tile sizes
    if st != fd.OK:
        raise fd.DecodeError(st, "batch_decode")
    log(f"[batch] autotuned in {time.time() - t1:.1f}s")

    def step():
        if fd.batch_decode(tups, ws, status=status, async_=True, graph=True) != fd.OK:
            raise fd.DecodeError(-1, "batch_decode")
    mean_s, per = _events_time(step, steps, warmup)
    if int(status[-1].item()) != fd.OK:
        raise fd.DecodeError(int(status[-1].item()), "batch_decode")
    # the same columns, one fd_decode call each (the single-column mode)
    wss = [fd.alloc_workspace(c.codec, t[1].numel(), c.n_strings) for c, t in zip(cols, tups)]

    def loop():
        for t, w in zip(tups, wss):
            if fd.decode_into(t[0], t[1], t[2], t[3], t[4], w, status=status[:1], async_=True) != fd.OK:
                raise fd.DecodeError(-1, "fd_decode")
    loop_s, _ = _events_time(loop, max(2, steps // 4), 1)
    bit_exact = None
    if check:
        ok = True
        for c, (out, out_off) in zip(cols, outs):
            ok &= bool(torch.equal(out.cpu(), torch.from_numpy(c.text)))
            ok &= bool(np.array_equal(out_off.cpu().numpy().astype(np.int64), c.text_off))
        bit_exact = ok
    B_alg = sum(algorithmic_bytes(c) for c in cols)
    # the bytes-weighted single-column reference: sum D / sum (D_j / single-column rate of its codec)
    if single_rates is None:
        single_rates = {"fsst8": single_rate("fsst_logs"), "onpair16": single_rate("onpair_urls")}
    ref = D / sum(c.decoded_bytes / single_rates[c.codec] for c in cols)
    res = {"value": round(D / mean_s / 1e9, 2), "decoded_bytes": int(D), "n_cols": n_cols,
           "single_column_reference_GBps": round(ref, 2), "batch_over_reference": round(D / mean_s / 1e9 / ref, 3),
           "single_column_GBps": {k: round(v, 2) for k, v in single_rates.items()},
           "ms_per_step": round(mean_s * 1e3, 4), "per_column_calls_GBps": round(D / loop_s / 1e9, 2),
           "batch_over_per_column": round(loop_s / mean_s, 3),
           "step_us": {"min": round(float(per.min()) * 1e6, 1), "p50": round(float(np.median(per)) * 1e6, 1)},
           "roofline": {"bound": "hbm", "achieved": round(B_alg / mean_s / 1e9, 1), "peak": HBM_PEAK_GBPS,
                        "unit": "GB/s", "frac": round(B_alg / mean_s / 1e9 / HBM_PEAK_GBPS, 4), "traffic": None,
                        "algorithmic_bytes": int(B_alg)},
           "bit_exact": bit_exact}
    if cpu:
        import oracle
        threads = max(1, min(16, os.cpu_count() or 1))
        sample = [c for c in cols if c.decoded_bytes <= (32 << 20)][:64]
        tot_t = tot_b = 0
        for c in sample:
            t_cpu, nb, _ = oracle.time_decode(c.codec, c.codes, c.code_off, c.dict_bytes, c.dict_lens,
                                              threads=threads, repeats=1)
            tot_t += t_cpu
            tot_b += nb
        res["cpu_baseline"] = {"value": round(tot_b / tot_t / 1e9, 3), "unit": "GB/s", "cores": threads,
                               "kind": "oracle", "sample": f"{len(sample)} columns of the batch "
                                                           f"({tot_b} decoded bytes), one pass"}
    log(f"[batch] {res['value']} GB/s (per-column calls {res['per_column_calls_GBps']} GB/s)")
    return res


def run_serve(seed: int | None, n_requests: int = 5000, load: float = 0.7, budget: int = 16 * 10**9,
              n_slots: int = 4, max_batch: int = 64, check: bool = True, n_chunks: int = 128,
              sat_load: float = 1.5, other_loads: tuple = (0.5, 0.9), single_rates: dict | None = None):
    """The served workload: Poisson arrivals at `load` x the server's measured
    batch capacity (latency at a moderate load), at each of `other_loads`, then
    at `sat_load` x capacity (offered above capacity: the served rate the server
    sustains).  Returns a result dict with p50 / p99 latency."""
    import gc
    import threading
    import numpy as np
    import torch
    import datagen
    import paper_2609_15034_amd as fd
    t0 = time.time()
    pool = datagen.serve_pool(seed=seed or 5, n_chunks=n_chunks)
    log(f"[serve] generated {len(pool.dicts)} dictionaries, {len(pool.chunks)} chunks "
        f"({sum(c.decoded_bytes for c in pool.chunks) / 1e6:.1f} MB) in {time.time() - t0:.1f}s")
    dev = torch.device("cuda")
    dicts = [fd.Dict(codec, torch.from_numpy(db).to(dev), torch.from_numpy(dl).to(dev))
             for codec, db, dl in pool.dicts]
    inputs = [_upload_column(c, dev) for c in pool.chunks]
    texts = [torch.from_numpy(c.text).to(dev) for c in pool.chunks] if check else None
    pool_bytes = sum(c.decoded_bytes for c in pool.chunks)
    # capacity: the whole pool as one batch, in the server's mode (three phases)
    tups = [(dicts[pool.chunk_dict[i]], inputs[i][0], inputs[i][1],
             torch.empty(c.n_strings + 1, dtype=inputs[i][1].dtype, device=dev),
             torch.empty(c.decoded_bytes, dtype=torch.uint8, device=dev)) for i, c in enumerate(pool.chunks)]
    tu = {"mode": 1, "tile_codes": 0, "grid": 0, "reserved": 0}
    ws = torch.empty(fd.batch_workspace_size(tups, tu), dtype=torch.uint8, device=dev)
    # (a hundred untimed batches first, about 0.1 s: the clocks settle, as they
    # have in the served runs that follow)
    cap_st = torch.zeros(len(tups) + 1, dtype=torch.int32, device=dev)
    cap_s, _ = _events_time(lambda: fd.batch_decode(tups, ws, tuning=tu, async_=True, status=cap_st), 20, 100)
    cap_bps = pool_bytes / cap_s
    # the same chunks one call each (no batching): the rate a request loop without batching reaches
    st1 = torch.zeros(1, dtype=torch.int32, device=dev)
    wss = [fd.alloc_workspace(c.codec, inputs[i][0].numel(), c.n_strings) for i, c in enumerate(pool.chunks)]

    def one_each():
        for i in range(len(pool.chunks)):
            fd.decode_into(tups[i][0], tups[i][1], tups[i][2], tups[i][3], tups[i][4], wss[i], status=st1,
                           async_=True)
    each_s, _ = _events_time(one_each, 3, 1)
    each_bps = pool_bytes / each_s
    del wss
    log(f"[serve] pool as one batch {cap_bps / 1e9:.1f} GB/s; one call per chunk {each_bps / 1e9:.1f} GB/s")

    def serve_once(ld, n_req, rseed):
        rng = np.random.default_rng(rseed)
        pick = rng.integers(0, len(pool.chunks), size=n_req)
        reqs = []
        for i in pick:
            c = pool.chunks[i]
            out = torch.empty(c.decoded_bytes, dtype=torch.uint8, device=dev)
            out_off = torch.empty(c.n_strings + 1, dtype=inputs[i][1].dtype, device=dev)
            reqs.append((dicts[pool.chunk_dict[i]], inputs[i][0], inputs[i][1], out_off, out))
        sizes = np.array([pool.chunks[i].decoded_bytes for i in pick], np.float64)
        rate = ld * cap_bps / sizes.mean()                        # requests per second
        gaps = rng.exponential(1.0 / rate, size=n_req)
        arrivals = np.cumsum(gaps) - gaps[0]
        log(f"[serve] load {ld}: offered {ld * cap_bps / 1e9:.1f} GB/s = {rate:.0f} requests/s")
        torch.cuda.synchronize()
        tickets = [0] * n_req
        lag = [0.0]
        sub_t = np.zeros(n_req)                                # submission times (s from the start)
        recs = [fd.Server.prepare(r) for r in reqs]          # built before the clock starts
        gc.disable()                                         # no collector pauses in the producer's schedule
        try:
            with fd.Server(max_inflight_bytes=budget, n_slots=n_slots, max_batch=max_batch) as srv:
                t_start = time.perf_counter()

                def producer():
                    for k in range(n_req):
                        dt = arrivals[k] - (time.perf_counter() - t_start)
                        if dt > 0:
                            time.sleep(dt)
                        else:
                            lag[0] = max(lag[0], -dt)
                        sub_t[k] = time.perf_counter() - t_start
                        tickets[k] = srv.submit(recs[k])
                th = threading.Thread(target=producer)
                th.start()
                th.join()
                res = [srv.wait(t) for t in tickets]
                wall = time.perf_counter() - t_start
                stats = srv.stats()
        finally:
            gc.enable()
        sts = np.array([r[0] for r in res])
        lat = np.array([r[1] for r in res]) / 1e3                    # ms
        if np.any(sts != 0):
            raise fd.DecodeError(int(sts[sts != 0][0]), "served decode")
        bit_exact = None
        if check:
            ok = True
            for k, i in enumerate(pick):
                ok &= bool(torch.equal(reqs[k][4], texts[i]))
            bit_exact = ok
        # steady window: drop the first 5% of requests (arrival times) from the rate and the latencies
        k0 = n_req // 20
        # a request completes at its submission plus its latency (the server's clock
        # runs from the submit call to the host seeing its batch done)
        completion = sub_t + lat / 1e3
        t_end = float(completion.max())
        D = float(sizes[k0:].sum())
        rate_window = t_end - float(arrivals[k0])
        # latency = completion - scheduled arrival (includes any lag of the producer behind the schedule)
        lat_sub = lat[k0:]
        lat = (completion - arrivals)[k0:] * 1e3
        out = {"value": round(D / rate_window / 1e9, 2), "unit": "GB/s", "n_requests": n_req,
               "steady_window": f"requests {k0}..{n_req - 1} (first 5% dropped)", "load": ld,
               "offered_GBps": round(ld * cap_bps / 1e9, 2),
               # the sampled arrivals' own rate over the window (Poisson noise around offered_GBps)
               "arrived_GBps": round(float(sizes[k0:-1].sum()) / max(float(arrivals[-1] - arrivals[k0]), 1e-9) / 1e9,
                                     2),
               "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                              "p99": round(float(np.percentile(lat, 99)), 3),
                              "mean": round(float(lat.mean()), 3), "max": round(float(lat.max()), 3),
                              "from": "scheduled arrival"},
               "latency_from_submit_ms": {"p50": round(float(np.percentile(lat_sub, 50)), 3),
                                          "p99": round(float(np.percentile(lat_sub, 99)), 3)},
               "mean_request_MB": round(float(sizes.mean()) / 1e6, 2),
               "max_inflight_bytes": stats["max_inflight_bytes"], "batches": stats["batches"],
               "mean_batch": round(stats["admitted"] / max(stats["batches"], 1), 2), "bit_exact": bit_exact,
               "producer_max_lag_ms": round(lag[0] * 1e3, 3), "wall_s": round(wall, 4)}
        log(f"[serve] load {ld}: {out['value']} GB/s, p50 {out['latency_ms']['p50']} ms, "
            f"p99 {out['latency_ms']['p99']} ms, mean batch {out['mean_batch']}, arrived {out['arrived_GBps']} GB/s, "
            f"submissions at most {out['producer_max_lag_ms']} ms behind their arrival times")
        return out

    if single_rates:
        # the bytes-weighted single-column reference of the pool (the 1 GiB columns' rates per codec)
        ref = pool_bytes / sum(c.decoded_bytes / single_rates[c.codec] / 1e9 for c in pool.chunks)
    out = serve_once(load, n_requests, (seed or 5) + 1)
    others = {}
    for k, ld in enumerate(other_loads):
        o = serve_once(ld, n_requests, (seed or 5) + 3 + k)
        others[str(ld)] = {key: o[key] for key in ("value", "offered_GBps", "arrived_GBps", "latency_ms", "mean_batch",
                                                   "bit_exact", "producer_max_lag_ms")}
    sat = serve_once(sat_load, n_requests, (seed or 5) + 2)
    out.update({"batch_capacity_GBps": round(cap_bps / 1e9, 2), "one_call_per_chunk_GBps": round(each_bps / 1e9, 2),
                "budget_bytes": budget, "slots": n_slots,
                "saturated": {k: sat[k] for k in ("value", "load", "offered_GBps", "latency_ms", "mean_batch",
                                                  "batches", "max_inflight_bytes", "bit_exact", "producer_max_lag_ms")},
                "saturated_over_capacity": round(sat["value"] * 1e9 / cap_bps, 3),
                "pool_stats": {codec: {"bytes_per_code": round(
                    sum(c.decoded_bytes for c in pool.chunks if c.codec == codec) /
                    max(1, sum(int(c.stats["n_codes"]) for c in pool.chunks if c.codec == codec)), 3)}
                    for codec in ("fsst8", "onpair16")},
                "other_loads": others})
    if single_rates:
        out["single_column_reference_GBps"] = round(ref / 1e9, 2)
        out["saturated_over_single_column"] = round(sat["value"] * 1e9 / ref, 3)
        out["capacity_over_single_column"] = round(cap_bps / ref, 3)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="fsst_logs_ngram", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=None)
    ap.add_argument("--mode", type=int, default=1, help="0 single pass (look-back), 1 three phases (default)")
    ap.add_argument("--tile-codes", type=int, default=0, help="codes per tile (0 = the largest)")
    ap.add_argument("--grid", type=int, default=0, help="workgroups (0 = all resident)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-check", action="store_true", help="skip the output check")
    ap.add_argument("--no-extra", action="store_true", help="default run: skip the batched and served legs")
    ap.add_argument("--sidecar", action="store_true",
                    help="decode with output positions from a stored sidecar (built once, before timing)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes (counter calibration) and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(the decode shards by contiguous string ranges with one int64 exchange per GPU; "
              "only the one-GPU kernel is built and measured)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2609_15034_amd as fd

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(2)
    fd.lib()  # fails loudly when the HIP library is not built

    if args.copy_calibration:
        gbps = copy_calibration(args.copy_calibration)
        print(json.dumps({"copy_bytes": args.copy_calibration, "copy_GBps": round(gbps, 1)}))
        return

    if args.workload in ("batch256", "serve"):
        if args.workload == "batch256":
            r = run_batch(args.steps, args.warmup, args.seed, check=not args.no_check, cpu=not args.no_cpu)
            cfg = {"workload": "batch256", "description": WORKLOADS["batch256"]["desc"],
                   "n_cols": r["n_cols"], "decoded_bytes": r["decoded_bytes"]}
            ms, steps, warmup = r["ms_per_step"], args.steps, args.warmup
        else:
            r = run_serve(args.seed, check=not args.no_check)
            cfg = {"workload": "serve", "description": WORKLOADS["serve"]["desc"], "n_requests": r["n_requests"],
                   "offered_GBps": r["offered_GBps"], "budget_bytes": r["budget_bytes"]}
            ms, steps, warmup = None, r["n_requests"], 0
        line = {"metric": METRIC, "value": r["value"], "unit": "GB/s", "n_gpus": 1, "steps": steps,
                "warmup": warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "dtype": "u8", "data": "synthetic", "config": cfg}
        line.update({k: v for k, v in r.items() if k not in ("value",)})
        print(json.dumps(line), flush=True)
        return

    t0 = time.time()
    col = make_column(args.workload, args.seed)
    log(f"[bench] generated {args.workload}: {col.stats} in {time.time() - t0:.1f}s")

    dev = torch.device("cuda")
    codes_np = col.codes.view(np.int16) if col.codec == "onpair16" else col.codes
    codes = torch.from_numpy(codes_np).to(dev)
    code_off = torch.from_numpy(col.code_off).to(dev)
    d = fd.Dict(col.codec, torch.from_numpy(col.dict_bytes).to(dev), torch.from_numpy(col.dict_lens).to(dev))
    D = col.decoded_bytes
    out = torch.empty(D, dtype=torch.uint8, device=dev)
    out_off = torch.empty(col.n_strings + 1, dtype=code_off.dtype, device=dev)
    tuning = {"mode": args.mode, "tile_codes": args.tile_codes, "grid": args.grid, "reserved": 0}
    ws = fd.alloc_workspace(col.codec, fd.codes_in(col.codec, codes), col.n_strings, tuning)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    sidecar = None
    if args.sidecar:                  # stored output positions, built once before timing
        if args.mode != 0:
            raise SystemExit("--sidecar decodes take mode 0 tuning")
        sidecar = fd.sidecar_build(d, codes, code_off, tuning)
    torch.cuda.synchronize()

    def step():
        if sidecar is not None:
            st = fd.decode_sidecar_into(d, codes, code_off, sidecar, out_off, out, ws, status=status, async_=True,
                                        tuning=tuning)
        else:
            st = fd.decode_into(d, codes, code_off, out_off, out, ws, status=status, async_=True, tuning=tuning)
        if st != fd.OK:
            raise fd.DecodeError(st)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if int(status.item()) != fd.OK:
        raise fd.DecodeError(int(status.item()))

    K = args.steps
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    # the dominant kernel (k_decode) timed inside the timed steps by the library's
    # own events on the stream it launches on
    fd.profile_begin(("decode",), K + 4)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    evs[0].record()
    for i in range(K):
        step()
        evs[i + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    prof = fd.profile_end()
    st = int(status.item())
    if st != fd.OK:
        raise fd.DecodeError(st)
    per = np.array([evs[i].elapsed_time(evs[i + 1]) / 1e3 for i in range(K)])   # seconds
    mean_s = float(per.mean())
    log(f"[bench] {K} steps: mean {mean_s * 1e6:.1f} us, min {per.min() * 1e6:.1f} us, "
        f"wall {wall / K * 1e6:.1f} us/step")

    bit_exact = None
    if not args.no_check and col.text is not None:
        ok_b = torch.equal(out, torch.from_numpy(col.text).to(dev))
        ok_o = torch.equal(out_off.to(torch.int64), torch.from_numpy(col.text_off).to(dev))
        bit_exact = bool(ok_b and ok_o)
        log(f"[bench] output vs source text: bytes {ok_b}, offsets {ok_o}")

    # every kernel of the step, timed over a few more steps (outside the timed region)
    fd.profile_begin(fd.PROF_KINDS, 64)
    for _ in range(5):
        step()
    torch.cuda.synchronize()
    per_kernel = fd.profile_end()

    B_alg = algorithmic_bytes(col) + (8 * sidecar.numel() if sidecar is not None else 0)
    value = D / mean_s / 1e9
    dec = prof["decode"]
    assert dec["launches"] == K and prof["dropped"] == 0, prof
    kern_s = dec["mean_us"] / 1e6
    achieved = B_alg / kern_s / 1e9
    src_hash = kernel_source_hash()
    tr = read_traffic(args.workload, src_hash) if sidecar is None else None
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": (int(tr["hbm_bytes_per_launch"]) if tr else None),
            "algorithmic_bytes": int(B_alg),
            "kernel": ("k_decode (expand, stored positions)" if sidecar is not None
                       else "k_decode (single pass)" if args.mode == 0 else "k_decode (expand)"),
            "duration_us": round(dec["mean_us"], 2),
            "duration_min_max_us": [round(dec["min_us"], 2), round(dec["max_us"], 2)],
            "step": {"achieved": round(B_alg / mean_s / 1e9, 1), "frac": round(B_alg / mean_s / 1e9 / HBM_PEAK_GBPS, 4),
                     "duration_us": round(mean_s * 1e6, 2)},
            "kernels_us": {k: round(v["mean_us"], 2) for k, v in per_kernel.items() if k != "dropped"}}
    log(f"[bench] k_decode mean {dec['mean_us']:.1f} us ({achieved:.0f} GB/s algorithmic), "
        f"kernels {roof['kernels_us']}")

    copy_gbps = copy_calibration(1 << 30, reps=3)

    cpu = None
    if not args.no_cpu:
        import oracle
        threads = max(1, min(16, os.cpu_count() or 1))
        times = []
        t_cpu, nb, ns = oracle.time_decode(col.codec, col.codes, col.code_off, col.dict_bytes, col.dict_lens,
                                           threads=threads, repeats=5, n_codes=int(col.stats["n_codes"]),
                                           times=times)
        # one thread on the first sixteenth of the strings
        n1 = max(1, ns // 16)
        t1, nb1, _ = oracle.time_decode(col.codec, col.codes, col.code_off, col.dict_bytes, col.dict_lens,
                                        threads=1, repeats=3, max_strings=n1, n_codes=int(col.stats["n_codes"]))
        cpu = {"value": round(nb / t_cpu / 1e9, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
               "sample": f"whole column ({nb} decoded bytes, {ns} strings), best of 5, {threads} threads on "
                         f"contiguous string-range shards",
               "median_GBps": round(nb / sorted(times)[len(times) // 2] / 1e9, 3),
               "single_thread": {"GBps": round(nb1 / t1 / 1e9, 3),
                                 "sample": f"the first {n1} strings ({nb1} decoded bytes), best of 3"},
               "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
        log(f"[bench] cpu oracle: {cpu['value']} GB/s on {threads} threads, "
            f"{cpu['single_thread']['GBps']} GB/s on one")

    res = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(mean_s * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload]["desc"],
                   "codec": col.codec, "decoded_bytes": D, "n_codes": int(col.stats["n_codes"]),
                   "n_strings": col.n_strings, "index_bits": 8 * col.code_off.dtype.itemsize,
                   "bytes_per_code": round(col.stats.get("bytes_per_code", 0.0), 3),
                   "escape_share": round(col.stats.get("escape_share", 0.0), 4),
                   "table": WORKLOADS[args.workload].get("table"),
                   "mode": args.mode, "tile_codes": args.tile_codes, "grid": args.grid,
                   "positions": positions_label(args.mode, sidecar is not None)},
        "decoded_frac_of_hbm_peak": round(value / HBM_PEAK_GBPS, 4),
        "step_us": {"min": round(float(per.min()) * 1e6, 2), "p50": round(float(np.median(per)) * 1e6, 2),
                    "p99": round(float(np.percentile(per, 99)) * 1e6, 2)},
        "copy_ceiling_GBps": round(copy_gbps, 1),
        "bit_exact": bit_exact,
        "roofline": roof,
        "cpu_baseline": cpu,
        "kernel_source_sha": src_hash,
    }
    if args.workload == "fsst_logs_ngram" and not args.no_extra:
        # the other columns, the small column's latency, the batched and served workloads (short runs)
        rates = {}
        try:
            rates["fsst8"] = single_rate("fsst_logs", mode=args.mode)     # the batch's FSST-8 recipe
            res["fsst_logs_GBps"] = round(rates["fsst8"], 2)
        except Exception as e:
            res["fsst_logs_GBps"] = {"error": f"{type(e).__name__}: {e}"}
        try:
            res["fsst_small"] = small_latency()
            res["fsst_small"]["three_phases_latency_us"] = small_latency(mode=1)["latency_us"]
        except Exception as e:
            res["fsst_small"] = {"error": f"{type(e).__name__}: {e}"}
        try:
            rates["onpair16"] = single_rate("onpair_urls", mode=args.mode)
            res["onpair_urls_GBps"] = round(rates["onpair16"], 2)
        except Exception as e:
            res["onpair_urls_GBps"] = {"error": f"{type(e).__name__}: {e}"}
        other = 1 - args.mode                           # the other way to the tile cursors
        key = "single_pass_GBps" if other == 0 else "three_phase_GBps"
        res[key] = {}
        for wl in ("fsst_logs_ngram", "fsst_logs", "onpair_urls"):
            try:
                res[key][wl] = round(single_rate(wl, mode=other), 2)
            except Exception as e:
                res[key][wl] = {"error": f"{type(e).__name__}: {e}"}
        for wl in ("onpair12_urls", "fsst12_logs"):     # 12-bit packed codes
            try:
                res[wl + "_GBps"] = round(single_rate(wl, mode=args.mode), 2)
            except Exception as e:
                res[wl + "_GBps"] = {"error": f"{type(e).__name__}: {e}"}
        # the batched and served legs first, on a fresh allocator (the legs after them hold large buffers)
        for key, fn in (("batch", lambda: run_batch(10, 2, None, check=not args.no_check, cpu=False,
                                                    single_rates=rates if len(rates) == 2 else None)),
                        ("serve", lambda: run_serve(None, n_requests=5000, check=not args.no_check,
                                                    single_rates=rates if len(rates) == 2 else None))):
            torch.cuda.empty_cache()
            try:
                res[key] = fn()
            except Exception as e:       # report, never lose the main line
                res[key] = {"error": f"{type(e).__name__}: {e}"}
        for key, fn in (("sidecar", sidecar_rates), ("take", take_rates)):
            res[key] = {}
            for wl in ("fsst_logs", "onpair_urls"):
                torch.cuda.empty_cache()
                try:
                    res[key][wl] = fn(wl)
                except Exception as e:
                    res[key][wl] = {"error": f"{type(e).__name__}: {e}"}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
