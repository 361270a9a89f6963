"""Autotuner of the batched form's grouped LU (run on the target GPU).

For every order bucket and precision it factors a synthetic batch under each
candidate configuration -- panel width 64 or 128, and the loop of the grouped
trailing update (four real products per complex step; three products with
operand pipelining; four products with operand pipelining) --
and writes the fastest per bucket to ``csrc/batch_tune.h``, which
``feast_batch_create`` consults (rebuild the library afterwards).

    python -m paper_1404_1768_amd.autotune [--out PATH] [--reps 3] [--summary PATH]

The factorisation time of a candidate is the time of ``invalidate + filter``
minus that of ``filter`` alone (the same grouped filter on cached factors),
the minimum over ``--reps`` repetitions.  The batches are random complex
matrices of orders drawn uniformly in each bucket (their LU costs what any
pencil of those orders costs: partial pivoting is value-independent work),
16 shifted systems per pencil, 16 right-hand sides.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))

# (lo, hi, pencils): orders drawn in [lo, hi); fewer pencils for larger orders
BUCKETS = [(64, 384, 48), (384, 768, 32), (768, 1536, 24), (1536, 3072, 12), (3072, 16385, 4)]
FP64, MIXED = 0, 1
# candidates: (panel width, opts.batch_update): 1 = four products, 2 = three
# products pipelined, 3 = four products pipelined
CANDIDATES = {FP64: [(64, 1), (64, 2), (64, 3), (128, 1), (128, 2), (128, 3)],
              MIXED: [(64, 1), (64, 2), (64, 3), (128, 1), (128, 2), (128, 3)]}
# batch_update value -> the library's feast::GROUP_* code
GROUP_CODE = {1: 0, 2: 1, 3: 2}


def _time_factor(fm, torch, ns, prec, nb, upd, As, Bs, Vs, reps):
    ms = [16] * len(ns)
    with fm.Batch(ns, ms, [0.0] * len(ns), [1.0] * len(ns), 16, prec=prec, nb=nb,
                  batch_update=upd) as b:
        b.filter(As, Bs, Vs)            # warm-up: factor, capture the graphs
        best_full = best_filter = float("inf")
        for _ in range(reps):
            b.invalidate()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b.filter(As, Bs, Vs)
            torch.cuda.synchronize()
            best_full = min(best_full, time.perf_counter() - t0)
            t0 = time.perf_counter()
            b.filter(As, Bs, Vs)
            torch.cuda.synchronize()
            best_filter = min(best_filter, time.perf_counter() - t0)
    return max(0.0, best_full - best_filter) * 1e3


def tune(reps: int = 3, seed: int = 1404):
    import numpy as np
    import torch
    import paper_1404_1768_amd as fm
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    rng = np.random.default_rng(seed)
    results = []
    for lo, hi, count in BUCKETS:
        hi_draw = min(hi, 4096)
        ns = sorted(int(x) for x in rng.integers(lo, hi_draw, count))
        gen.manual_seed(seed + lo)
        As = [torch.randn((n, n), dtype=torch.complex128, device=dev, generator=gen) for n in ns]
        Bs = [torch.randn((n, n), dtype=torch.complex128, device=dev, generator=gen) for n in ns]
        Vs = [torch.randn((n, 16), dtype=torch.complex128, device=dev, generator=gen) for n in ns]
        for prec in (FP64, MIXED):
            times = {}
            for nb, upd in CANDIDATES[prec]:
                t = _time_factor(fm, torch, ns, prec, nb, upd, As, Bs, Vs, reps)
                times["nb%d_u%d" % (nb, upd)] = round(t, 3)
                print("[autotune] orders %d..%d (%d pencils) %s nb=%d update=%d: %.2f ms" %
                      (lo, hi, count, "fp64" if prec == FP64 else "mixed", nb, upd, t),
                      file=sys.stderr, flush=True)
            key = min(times, key=times.get)
            nb, upd = (int(x) for x in key[2:].split("_u"))
            results.append({"lo": lo, "hi": hi, "prec": prec, "nb": nb, "update": GROUP_CODE[upd],
                            "orders": ns, "ms": times})
        del As, Bs, Vs
        torch.cuda.empty_cache()
    return results


def write_header(results, path, device):
    lines = [
        "// Configurations of the batched form's grouped LU, per precision and order",
        "// bucket: the panel width and the loop of the trailing update (feast::GROUP_*).",
        "// Written by `python -m paper_1404_1768_amd.autotune` from factorisation",
        "// timings of every candidate on %s; entries are looked up with the order" % device,
        "// n* that splits a batch's LU work in half.",
        "#pragma once",
        "#include <cstdint>",
        "",
        "namespace feast_tune {",
        "",
        "struct Entry {",
        "  int64_t lo, hi;  // bucket: lo <= n* < hi",
        "  int prec;        // FEAST_FP64 or FEAST_MIXED",
        "  int nb;          // panel width, 64 or 128",
        "  int update;      // feast::GROUP_PLAIN, GROUP_UPDATE_M3 or GROUP_UPDATE_PIPE",
        "};",
        "",
        "inline constexpr Entry kBatch[] = {",
    ]
    for r in results:
        ms = ", ".join("%s %.2f" % (k, v) for k, v in sorted(r["ms"].items()))
        lines.append("    {%d, %d, %d, %d, %d},  // ms: %s" % (r["lo"], r["hi"], r["prec"], r["nb"],
                                                            r["update"], ms))
    lines += ["};", "", "}  // namespace feast_tune", ""]
    with open(path, "w") as f:
        f.write("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "csrc", "batch_tune.h"))
    ap.add_argument("--summary", default=None, help="also write the timings as JSON here")
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    import torch
    props = torch.cuda.get_device_properties(0)
    device = "%s (%s)" % (props.name, getattr(props, "gcnArchName", "?"))
    results = tune(args.reps)
    write_header(results, args.out, device)
    if args.summary:
        with open(args.summary, "w") as f:
            json.dump({"device": device, "buckets": results}, f, indent=1)
    print("[autotune] wrote %s" % args.out, file=sys.stderr)


if __name__ == "__main__":
    main()
