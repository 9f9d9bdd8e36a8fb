"""HBM traffic of the sweep kernel from two rocprofv3 counter runs.

rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE each write a counter_collection.csv
with one row per dispatch (KiB per dispatch). The run that is measured also launches
the library's copy kernel on a buffer of known size (4 GiB read, 4 GiB written); the
ratio of those known bytes to what each counter reads for the copy kernel is the
scale factor applied to the sweep's readings. The result is written as JSON keyed by
a hash of the sweep's sources, so that a reader can tell whether the counters were
taken on the kernel as it now stands.

Usage: python -m paper_2606_00641_amd.pmc_traffic --fetch F.csv --write W.csv
       --key resistive_256/f32 --cells N --bytes-per-cell B --out traffic.json
       [--kernel sweep|pair|pair_body] [--store-cells M] [--merge]
--kernel pair takes the FP16/BF16 two-cells-per-lane sweep (k_sweep2) of a periodic
lattice instead of the plain one-cell sweep, pair_body its form on the open lattice
with the homogenized body, which loads every cell but stores nothing for the cells of
the body's box (--store-cells: the cells it stores); --merge adds the record to an
existing file taken on the same sources.
"""
import argparse
import csv
import hashlib
import json
import os
import re

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
SWEEP_SOURCES = ("vlbm_device.h", "vlbm_kernels.h", "vlbm_physics.h", "vlbm_sweep.hip")
COPY_BYTES = 4 << 30


_COMMENT = re.compile(r"//[^\n]*|/\*.*?\*/", re.S)


def kernel_source_hash():
    """Hash of the code the sweep kernel is built from: its sources with the comments
    taken out and the whitespace collapsed, so that a change of a comment leaves it."""
    h = hashlib.sha256()
    for name in SWEEP_SOURCES:
        with open(os.path.join(CSRC, name), encoding="utf-8") as fh:
            code = " ".join(_COMMENT.sub(" ", fh.read()).split())
        h.update(name.encode())
        h.update(code.encode())
    return h.hexdigest()[:16]


def read_counter(path, counter):
    """[(kernel name, KiB)] in dispatch order for one counter."""
    rows = []
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] == counter:
                rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return rows


SWEEP_RE = re.compile(r"k_sweep<(\d+), (\d+), (\d+), (\d+), (\d+), (\d+)((?:, (?:true|false|\d+))*)>")


def per_parity(rows, st, d, model):
    """Mean KiB per dispatch of the plain periodic BGK sweep for each parity (no
    injection, no face or exchange variant)."""
    acc = {}
    for name, v in rows:
        m = SWEEP_RE.search(name)
        if not m:
            continue
        ST, D, MODEL, PAR, BODY, COLL, flags = m.groups()
        if (int(ST), int(D), int(MODEL), int(BODY), int(COLL)) != (st, d, model, 0, 0) or "true" in flags \
                or re.search(r", [1-9]", flags):
            continue
        acc.setdefault(int(PAR), []).append(v)
    return {p: sum(v) / len(v) for p, v in sorted(acc.items())}


PAIR_RE = re.compile(r"k_sweep2<(\d+), (\d+), (\d+), (\d+), (\d+), (true|false), (true|false)>")


def per_parity_pair(rows, st, d, model, body=False):
    """Mean KiB per dispatch of the two-cells-per-lane BGK sweep for each parity: the
    plain periodic one, or (body) the one of an open lattice with the homogenized body
    (x faces in the sweep, the body's box left to the box sweep)."""
    acc = {}
    for name, v in rows:
        m = PAIR_RE.search(name)
        if not m:
            continue
        ST, D, MODEL, PAR, COLL = (int(x) for x in m.groups()[:5])
        flags = m.groups()[5:]
        if (ST, D, MODEL, COLL) != (st, d, model, 0) or flags != (("true", "true") if body else ("false", "false")):
            continue
        acc.setdefault(PAR, []).append(v)
    return {p: sum(v) / len(v) for p, v in sorted(acc.items())}


def copy_kib(rows):
    vals = [v for name, v in rows if name.startswith("k_copy") or " k_copy(" in name or "::k_copy(" in name]
    if not vals:
        raise SystemExit("no copy-kernel dispatch in the counter file")
    return sum(vals) / len(vals)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--key", default="resistive_256/f32")
    ap.add_argument("--storage", type=int, default=1, help="storage code of the sweep (1 = FP32)")
    ap.add_argument("--dim-code", type=int, default=3, help="lattice code of the sweep (3 = D3Q7)")
    ap.add_argument("--model", type=int, default=1, help="model code (1 = resistive)")
    ap.add_argument("--cells", type=int, required=True)
    ap.add_argument("--bytes-per-cell", type=int, required=True)
    ap.add_argument("--commands", nargs="*", default=[])
    ap.add_argument("--store-cells", type=int, default=None,
                    help="cells whose populations the kernel stores (default --cells; the body form stores "
                         "nothing for the cells of the body's box)")
    ap.add_argument("--kernel", choices=("sweep", "pair", "pair_body"), default="sweep")
    ap.add_argument("--merge", action="store_true", help="add the record to an existing --out file")
    ap.add_argument("--out", required=True)
    args = ap.parse_args()

    fr = read_counter(args.fetch, "FETCH_SIZE")
    wr = read_counter(args.write, "WRITE_SIZE")
    cf, cw = copy_kib(fr), copy_kib(wr)
    fetch_factor = COPY_BYTES / (cf * 1024.0)
    write_factor = COPY_BYTES / (cw * 1024.0)
    if args.kernel == "sweep":
        select = per_parity
    else:
        def select(rows, st, d, model):
            return per_parity_pair(rows, st, d, model, body=args.kernel == "pair_body")
    pf = select(fr, args.storage, args.dim_code, args.model)
    pw = select(wr, args.storage, args.dim_code, args.model)
    if not pf or set(pf) != set(pw):
        raise SystemExit(f"sweep dispatches missing: fetch parities {sorted(pf)}, write parities {sorted(pw)}")
    fetch_b = sum(pf.values()) / len(pf) * 1024.0 * fetch_factor
    write_b = sum(pw.values()) / len(pw) * 1024.0 * write_factor
    store_cells = args.cells if args.store_cells is None else args.store_cells
    algo = (args.cells + store_cells) * args.bytes_per_cell // 2
    kname = "k_sweep" if args.kernel == "sweep" else "k_sweep2 (two cells per lane)"
    form = "homogenized body outside its box, x faces" if args.kernel == "pair_body" else "no body"
    rec = {
        "kernel": f"{kname}<storage {args.storage}, lattice {args.dim_code}, model {args.model}, parity, {form}, BGK>",
        "per_parity_raw_kib": {str(p): {"fetch_kib": pf[p], "write_kib": pw[p]} for p in pf},
        "fetch_bytes_per_launch": round(fetch_b),
        "write_bytes_per_launch": round(write_b),
        "bytes_per_launch": round(fetch_b + write_b),
        "algorithmic_bytes_per_launch": algo,
        "cells_loaded": args.cells,
        "cells_stored": store_cells,
        "ratio_to_algorithmic": round((fetch_b + write_b) / algo, 4),
    }
    rec["copy_kernel"] = {"FETCH_SIZE_kib": cf, "WRITE_SIZE_kib": cw, "fetch_factor": round(fetch_factor, 5),
                          "write_factor": round(write_factor, 5)}
    rec["commands"] = args.commands
    if args.merge:
        with open(args.out) as fh:
            out = json.load(fh)
        if out.get("kernel_hash") != kernel_source_hash():
            raise SystemExit("--merge: the existing file was taken on other sources")
        out["records"][args.key] = rec
        with open(args.out, "w") as fh:
            json.dump(out, fh, indent=1)
        print(json.dumps(rec))
        return
    out = {
        "description": "HBM traffic of the benchmark's dominant kernel from two rocprofv3 --pmc runs "
                       "(FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by the ratio of the known "
                       "bytes of the library's copy kernel (4 GiB read, 4 GiB written) to what the same counter "
                       "reads for it.",
        "commands": args.commands,
        "copy_kernel": {"bytes_read": COPY_BYTES, "bytes_written": COPY_BYTES, "FETCH_SIZE_kib": cf,
                        "WRITE_SIZE_kib": cw, "fetch_factor": round(fetch_factor, 5),
                        "write_factor": round(write_factor, 5)},
        "kernel_hash_sources": list(SWEEP_SOURCES),
        "kernel_hash": kernel_source_hash(),
        "records": {args.key: rec},
    }
    with open(args.out, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
