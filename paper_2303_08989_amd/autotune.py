"""Tile autotuner of the panel GEMM (64 x 64 vs 128 x 128 outputs per
workgroup), run on the GPU.

For a set of GEMM shapes -- the standalone CGEMM sizes and the matrix-core
GEMMs of the batched sliced-network pass (each with its batch count), and
the groups of them that run as one grouped launch -- and for the FP16X2,
BF16X3 and FP32 kernels, it times both tiles (hipEvents,
median of repetitions, a 512 MiB buffer write before each so that operands
are not served from the Infinity Cache), then writes

* ``tile_table.inc``: rules by the number of 128 x 128 output tiles over all
  batch entries and group entries (power-of-two buckets): each bucket takes the tile with the
  smaller summed time over its shapes and modes; consecutive buckets with
  the same tile merge.  The library compiles it in (``gemm_tile``).
* ``autotune.json``: every timing.

Usage (GPU): ``python -m paper_2303_08989_amd.autotune --out DIR``; copy
DIR/tile_table.inc to csrc/ and rebuild.
"""
import argparse
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

# (m, n, k, batch): standalone sizes, then the matrix-core GEMMs of the
# batched pass of the 53-qubit network (2^18 intermediates, 1024 slices)
DEFAULT_SHAPES = [
    (512, 512, 512, 1), (768, 768, 768, 1), (1024, 1024, 1024, 1), (1536, 1536, 1536, 1),
    (2048, 2048, 2048, 1), (4096, 4096, 4096, 1), (8192, 8192, 8192, 1),
    (8192, 256, 32, 1), (512, 16384, 64, 1), (512, 256, 128, 1), (1024, 2048, 128, 1),
    (1024, 512, 2048, 1), (2048, 512, 256, 1), (1024, 128, 2048, 1), (128, 4096, 512, 2),
    (4096, 4096, 64, 4),
]
# groups of uneven GEMMs run as one grouped launch: the tree levels of that
# batched pass with more than one matrix-core GEMM
DEFAULT_GROUPS = [
    [(8192, 256, 32), (512, 16384, 64), (512, 256, 128)],
    [(1024, 2048, 128), (1024, 512, 2048)],
    [(2048, 512, 256), (1024, 128, 2048)],
]
MODES = ("fp16x2", "bf16x3", "fp32")


def _bucket(tiles128):
    return 0 if tiles128 <= 1 else int(math.floor(math.log2(tiles128)))


def _tiles128(shapes):
    return sum(-(-m // 128) * -(-n // 128) * b for (m, n, k, b) in shapes)


def measure(shapes, reps=10, groups=()):
    import torch
    import paper_2303_08989_amd as qce
    h = qce.Handle(0)
    flush = torch.empty(512 << 18, dtype=torch.float32, device="cuda")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g = torch.Generator(device="cuda").manual_seed(5)
    rows = []
    for (m, n, k, batch) in shapes:
        A = torch.randn(batch * m * k, dtype=torch.complex64, device="cuda", generator=g)
        B = torch.randn(batch * k * n, dtype=torch.complex64, device="cuda", generator=g)
        C = torch.empty(batch * m * n, dtype=torch.complex64, device="cuda")
        for mode in MODES:
            h.set_mode(mode)
            rec = {"m": m, "n": n, "k": k, "batch": batch, "mode": mode}
            for tile in (64, 128):
                h.set_gemm_tile(tile)

                def call():
                    qce.cgemm_strided_batched(h, "N", "N", m, n, k, A, m, m * k, B, k, k * n, C, m, m * n, batch)
                for _ in range(2):
                    call()
                ts = []
                for r in range(reps):
                    flush.fill_(float(r))
                    ev0.record()
                    call()
                    ev1.record()
                    ev1.synchronize()
                    ts.append(ev0.elapsed_time(ev1))
                rec[f"ms_{tile}"] = float(np.median(ts))
            rec["tiles128"] = _tiles128([(m, n, k, batch)])
            rec["chunks"] = -(-k // 16)
            rows.append(rec)
            print(json.dumps(rec), flush=True)
        del A, B, C
    for grp in groups:
        bufs = []
        for (m, n, k) in grp:
            bufs.append((torch.randn(m * k, dtype=torch.complex64, device="cuda", generator=g),
                         torch.randn(k * n, dtype=torch.complex64, device="cuda", generator=g),
                         torch.empty(m * n, dtype=torch.complex64, device="cuda")))
        descs = [{"m": m, "n": n, "k": k, "A": A, "lda": m, "B": B, "ldb": k, "C": C, "ldc": m}
                 for (m, n, k), (A, B, C) in zip(grp, bufs)]
        for mode in MODES:
            h.set_mode(mode)
            rec = {"group": [list(x) for x in grp], "mode": mode,
                   "tiles128": _tiles128([(m, n, k, 1) for (m, n, k) in grp]),
                   "chunks": max(-(-k // 16) for (m, n, k) in grp)}
            for tile in (64, 128):
                h.set_gemm_tile(tile)
                for _ in range(2):
                    qce.cgemm_grouped(h, descs)
                ts = []
                for r in range(reps):
                    flush.fill_(float(r))
                    ev0.record()
                    qce.cgemm_grouped(h, descs)
                    ev1.record()
                    ev1.synchronize()
                    ts.append(ev0.elapsed_time(ev1))
                rec[f"ms_{tile}"] = float(np.median(ts))
            rows.append(rec)
            print(json.dumps(rec), flush=True)
        del bufs, descs
    h.set_gemm_tile(0)
    h.close()
    return rows


# k classes of the table: fewer than LONG_K_CHUNKS chunks of 16 k-values
# (output-dominated GEMMs) and the rest
LONG_K_CHUNKS = 16


def table(rows):
    """Rules (min_tiles128, min_chunks, tile) from the timings: one rule per
    measured power-of-two bucket of 128 x 128 tiles and k class (short or
    long k), each taking the tile with the smaller summed median time over
    its shapes and modes, listed in ascending order so that the last rule
    whose thresholds a GEMM reaches is its own bucket's.  A bucket with only
    one k class measured uses that class's tile for both."""
    sums = {}
    for r in rows:
        key = (_bucket(r["tiles128"]), LONG_K_CHUNKS if r.get("chunks", 0) >= LONG_K_CHUNKS else 0)
        s = sums.setdefault(key, [0.0, 0.0])
        s[0] += r["ms_64"]
        s[1] += r["ms_128"]
    rules = []
    for b in sorted({k[0] for k in sums}):
        lo = 0 if b == 0 else 1 << b
        best = {c: (64 if sums[(b, c)][0] < sums[(b, c)][1] else 128) for c in (0, LONG_K_CHUNKS) if (b, c) in sums}
        for c in (0, LONG_K_CHUNKS):
            rules.append((lo, c, best.get(c, next(iter(best.values())))))
    if rules:
        rules[0] = (0,) + tuple(rules[0][1:])
        if len(rules) > 1 and rules[1][0] != 0 and rules[0][1] == 0 and rules[1][1] != 0:
            rules[1] = (0,) + tuple(rules[1][1:])
    return rules, {f"{b}/{c}": v for (b, c), v in sums.items()}


def write_table(rules, path):
    lines = [
        "// Tile shape of the panel GEMM by output size, written by",
        "// paper_2303_08989_amd/autotune.py from timings of both tiles (the summed",
        "// median time over the measured shapes and modes of each power-of-two",
        "// bucket of 128 x 128 output tiles, batch entries included, and k class).",
        "// { first count of 128 x 128 tiles (all batch entries), first chunk count",
        "//   (k / 16), tile }: the last rule whose firsts are both reached applies.",
        "static const TileRule kTileRules[] = {",
    ]
    lines += [f"    {{{lo}, {ch}, {tile}}}," for lo, ch, tile in rules]
    lines.append("};")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="gpurun_out/autotune")
    ap.add_argument("--reps", type=int, default=10)
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    rows = measure(DEFAULT_SHAPES, args.reps, DEFAULT_GROUPS)
    rules, sums = table(rows)
    write_table(rules, os.path.join(args.out, "tile_table.inc"))
    with open(os.path.join(args.out, "autotune.json"), "w") as f:
        json.dump({"rows": rows, "bucket_ms_64_128": sums, "rules": rules}, f, indent=1)
    print("rules:", rules, file=sys.stderr)


if __name__ == "__main__":
    main()
