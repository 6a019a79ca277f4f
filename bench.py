#!/usr/bin/env python3
"""Decode throughput of one MI355X on a synthetic string column.

A step is one full decode of the column (the whole hot path: workspace reset,
code load, escape parity, decoded-length scan, tile cursors by look-back,
LDS assembly, 16-byte drain, Arrow offsets) with every input resident in HBM
and the dictionary prepared beforehand (the paper repacks dictionaries before
timing).  Default workload: FSST-8 log lines, 1 GiB decoded, int64 offsets.

Prints one JSON line:
  value        decoded GB/s (1e9 output bytes per second) = decoded bytes /
               mean step time
  roofline     algorithmic bytes (decoded bytes + code bytes + code offsets read
               + Arrow offsets written + dictionary) / mean step time, against
               the 8 TB/s HBM peak; `traffic` is the HBM bytes per launch from
               the committed rocprofv3 counter summary when it was taken on the
               current kernel source, else null
  cpu_baseline the CPU oracle on this host's cores over the same column
  bit_exact    GPU output == the generated source text (bytes and offsets)

  python bench.py [--workload fsst_logs|onpair_urls|fsst_small] [--steps K] [--warmup W]
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
WORKLOADS = {
    "fsst_logs": dict(codec="fsst8", desc="FSST-8 log lines, 1 GiB decoded, int64 offsets"),
    "onpair_urls": dict(codec="onpair16", desc="OnPair-16 URL/identifier strings, 1 GiB decoded, int64 offsets"),
    "fsst_small": dict(codec="fsst8", desc="FSST-8 printable strings, 10,000 strings, int32 offsets"),
}
KERNEL_SOURCES = ["paper_2609_15034_amd/csrc/fd_kernels.hip", "paper_2609_15034_amd/csrc/fd_internal.h",
                  "paper_2609_15034_amd/csrc/fd_host.cpp"]


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
    if name == "fsst_logs":
        return datagen.fsst_logs(seed=seed or 2)
    if name == "onpair_urls":
        return datagen.onpair_urls(seed=seed or 3)
    if name == "fsst_small":
        return datagen.fsst_small(seed=seed or 1)
    raise ValueError(name)


def algorithmic_bytes(col) -> int:
    """Bytes the decode must move at minimum: write the decoded bytes, read the
    codes of the decoded range, read the code offsets, write the Arrow offsets,
    read the dictionary once."""
    n_used = int(col.code_off[-1] - col.code_off[0])
    code_bytes = 1 if col.codec == "fsst8" else 2
    w_off = col.code_off.dtype.itemsize
    return (col.decoded_bytes + n_used * code_bytes + 2 * (col.n_strings + 1) * w_off
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


def read_traffic(workload: str, src_hash: str):
    path = os.path.join(ROOT, "profiles", f"decode_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha") != src_hash:
        return None
    return t


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="fsst_logs", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=None)
    ap.add_argument("--mode", type=int, default=0, help="0 single pass (look-back), 1 three phases")
    ap.add_argument("--sb", type=int, default=0, help="strings per tile (0 = automatic)")
    ap.add_argument("--grid", type=int, default=0, help="workgroups (0 = all resident)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-check", action="store_true", help="skip the output check")
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

    t0 = time.time()
    col = make_column(args.workload, args.seed)
    log(f"[bench] generated {args.workload}: {col.stats} in {time.time() - t0:.1f}s")

    dev = torch.device("cuda")
    codes_np = col.codes if col.codec == "fsst8" else col.codes.view(np.int16)
    codes = torch.from_numpy(codes_np).to(dev)
    code_off = torch.from_numpy(col.code_off).to(dev)
    d = fd.Dict(col.codec, torch.from_numpy(col.dict_bytes).to(dev), torch.from_numpy(col.dict_lens).to(dev))
    D = col.decoded_bytes
    out = torch.empty(D, dtype=torch.uint8, device=dev)
    out_off = torch.empty(col.n_strings + 1, dtype=code_off.dtype, device=dev)
    tuning = {"mode": args.mode, "strings_per_tile": args.sb, "grid": args.grid, "reserved": 0}
    ws = fd.alloc_workspace(col.codec, codes.numel(), col.n_strings, tuning)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()

    def step():
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
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    evs[0].record()
    for i in range(K):
        step()
        evs[i + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
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

    B_alg = algorithmic_bytes(col)
    value = D / mean_s / 1e9
    achieved = B_alg / mean_s / 1e9
    src_hash = kernel_source_hash()
    tr = read_traffic(args.workload, src_hash)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": (int(tr["hbm_bytes_per_launch"]) if tr else None),
            "algorithmic_bytes": int(B_alg), "kernel": "k_decode (single pass) + k_reset",
            "duration_us": round(mean_s * 1e6, 2)}

    copy_gbps = copy_calibration(1 << 30, reps=3)

    cpu = None
    if not args.no_cpu:
        import oracle
        threads = max(1, min(16, os.cpu_count() or 1))
        t_cpu, nb, ns = oracle.time_decode(col.codec, col.codes, col.code_off, col.dict_bytes, col.dict_lens,
                                           threads=threads, repeats=3)
        cpu = {"value": round(nb / t_cpu / 1e9, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
               "sample": f"whole column ({nb} decoded bytes, {ns} strings), best of 3, {threads} threads on "
                         f"contiguous string-range shards"}
        log(f"[bench] cpu oracle: {cpu['value']} GB/s on {threads} threads")

    res = {
        "metric": "decoded GB/s per GPU (fraction of HBM peak), bit-exact",
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
                   "mode": args.mode, "strings_per_tile": args.sb, "grid": args.grid},
        "decoded_frac_of_hbm_peak": round(value / HBM_PEAK_GBPS, 4),
        "step_us": {"min": round(float(per.min()) * 1e6, 2), "p50": round(float(np.median(per)) * 1e6, 2),
                    "p99": round(float(np.percentile(per, 99)) * 1e6, 2)},
        "copy_ceiling_GBps": round(copy_gbps, 1),
        "bit_exact": bit_exact,
        "roofline": roof,
        "cpu_baseline": cpu,
        "kernel_source_sha": src_hash,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
