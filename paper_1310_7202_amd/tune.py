"""Autotuner of the grouped products of rlu_factor_batched.

    python -m paper_1310_7202_amd.tune [--count 256] [--write]

For each of the five products of the batched form (sketch, Gram matrix,
projection, S^{-1} C, L = Lv L_b) and each storage type (FP64, FP32), times
the product's phase over a batch of uneven problems (m, n ~ U[256, 4096],
rank r ~ U[8, 64], k = r, l = r + 8) with every compiled tile shape, and
keeps the fastest.  With --write the result replaces csrc/tuned_tiles.h
(rebuild the library afterwards).  Needs a GPU; the batch is generated on it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

PHASES = ["sketch_gemm", "gram_gemm", "project_gemm", "solve_gemm", "form_l_gemm"]
HEADER = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "tuned_tiles.h")


def _batch(torch, count, seed, dtype):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import workloads

    shapes = workloads.batch_shapes(count, seed=seed)
    items = []
    for i, (m, n, r, s) in enumerate(shapes):
        A = workloads.low_rank_plus_noise_torch(m, n, r, 1e-6, s, dtype=dtype)
        items.append((A, r, r + 8, 7000 + i))
    torch.cuda.synchronize()
    return items


def tune(count=256, seed=104, reps=3, log=print):
    import torch
    import paper_1310_7202_amd as rlu

    names = rlu.tile_names()
    result = {}
    for storage, dtype, prec in ((0, torch.float64, rlu.PREC_FP64),
                                 (1, torch.float32, rlu.PREC_FP32)):
        items = _batch(torch, count, seed, dtype)
        h = rlu.Handle(0)
        h.set_timing(True)
        batch = rlu.Batch(items, precision=prec)
        batch.run(h)                          # warm-up
        torch.cuda.synchronize()
        for p, phase in enumerate(PHASES):
            times = {}
            for cfg in names:
                h.set_tile(p, cfg)
                best = float("inf")
                for _ in range(reps):
                    batch.run(h)
                    torch.cuda.synchronize()
                    best = min(best, h.phase_times(0)[phase])
                times[cfg] = best
            h.set_tile(p, -1)
            pick = min(times, key=times.get)
            result[(p, storage)] = (pick, times)
            log(f"storage {'FP64' if storage == 0 else 'FP32'} {phase}: "
                + ", ".join(f"{names[c]} {t:.3f}" for c, t in sorted(times.items()))
                + f" -> {names[pick]}")
        h.close()
        del batch, items
        torch.cuda.empty_cache()
    return result, names


def write_header(result, names, count, path=HEADER):
    rows = []
    for p in range(5):
        rows.append("{" + ", ".join(str(result[(p, s)][0]) for s in (0, 1)) + "}")
    record = []
    for (p, s), (pick, times) in sorted(result.items()):
        record.append(f"//   {PHASES[p]:<13} {'FP64' if s == 0 else 'FP32'}: "
                      + ", ".join(f"{names[c]} {t:.3f}" for c, t in sorted(times.items()))
                      + f"  -> {names[pick]}")
    text = f"""// Tile shapes of the grouped products of the batched form, written by
// paper_1310_7202_amd/tune.py from timings on MI355X (see the record below).
// kGroupedTile[product][storage]: product 0 sketch, 1 Gram, 2 projection,
// 3 S^{{-1}} C, 4 L = Lv L_b; storage 0 FP64, 1 FP32.  -1 keeps the built-in
// rule (a tile at least as wide as l for the sketch, 64 x 64 otherwise).
//
// Record: phase time (ms, best of 3) of a batch of {count} problems (m, n ~
// U[256, 4096], r ~ U[8, 64], k = r, l = r + 8) per tile shape:
{chr(10).join(record)}
#pragma once

namespace rlu {{
namespace tuned {{

constexpr int kGroupedTile[5][2] = {{{", ".join(rows)}}};

}}  // namespace tuned
}}  // namespace rlu
"""
    with open(path, "w") as f:
        f.write(text)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--count", type=int, default=256)
    ap.add_argument("--seed", type=int, default=104)
    ap.add_argument("--write", action="store_true", help="rewrite csrc/tuned_tiles.h")
    ap.add_argument("--header", default=HEADER, help="where --write puts the table")
    ap.add_argument("--json", default=None, help="also write the timings as JSON here")
    args = ap.parse_args()
    import torch

    if not torch.cuda.is_available():
        print("tune needs a GPU", file=sys.stderr)
        sys.exit(2)
    result, names = tune(args.count, args.seed, log=lambda s: print(s, flush=True))
    if args.json:
        with open(args.json, "w") as f:
            json.dump({f"{PHASES[p]}/{'fp64' if s == 0 else 'fp32'}":
                       {names[c]: t for c, t in times.items()} | {"pick": names[pick]}
                       for (p, s), (pick, times) in result.items()}, f, indent=1)
    if args.write:
        write_header(result, names, args.count, args.header)
        print(f"wrote {args.header}")


if __name__ == "__main__":
    main()
