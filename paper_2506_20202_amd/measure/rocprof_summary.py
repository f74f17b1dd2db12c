"""Summaries of rocprofv3 CSV output (--output-format csv) as short markdown.

  trace DIR [--first NAME]             per-kernel dispatches and mean duration
  pmc DIR [--first NAME]               per-kernel counter values per dispatch
  hbm FETCH_DIR WRITE_DIR [--first NAME] [--sources F ...]
                                       HBM bytes per dispatch from a FETCH_SIZE
                                       run and a WRITE_SIZE run, scaled by what
                                       the same counters read for the plain
                                       256 MiB device copy that
                                       ``bench.py --calibrate-copy`` adds

Only the dispatches of the profiled frames are summarised: from the launch
of the preprocess kernel right before the first dispatch whose name contains
NAME (default ``blend_kernel``; ``__all__`` keeps every dispatch).  Options:
--title and --command are written into the header, --out writes the summary
to a file as well.  Kernel names are shortened (namespaces and argument lists
dropped) and kept apart by grid size.  A measurement tool, not part of the
rendering path.
"""
import argparse
import csv
import glob
import hashlib
import os
import sys
from collections import defaultdict

COPY_BYTES = 256 << 20


def _rows(d, suffix):
    out = []
    for f in sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)):
        with open(f) as fh:
            out += list(csv.DictReader(fh))
    return out


def _col(r, *names):
    for n in names:
        if n in r:
            return r[n]
    raise KeyError(names)


def short(name):
    n = name.replace("(anonymous namespace)::", "").replace("rara::", "")
    depth = 0
    for i, ch in enumerate(n):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            n = n[:i]
            break
    if n.startswith("void "):
        n = n[5:]
    return n[:90]


def _is_copy(name):
    return "copyBuffer" in name or "direct_copy" in name


def _region_start(dispatches, marker):
    """First dispatch id of the profiled frames: the preprocess launch right
    before the first dispatch whose name holds ``marker``."""
    if marker == "__all__":
        return 0
    ids = sorted(dispatches)
    first = next((i for i, n in ids if marker in n), None)
    if first is None:
        return 0
    pre = [i for i, n in ids if i < first and "preprocess" in n]
    return pre[-1] if pre else first


def _header(args, what):
    lines = [f"# {args.title or what}", ""]
    if args.command:
        lines += ["Command (from the repository root on one MI355X, after `cd /tmp && export TMPDIR=/tmp`):", ""]
        lines += [f"    {c}" for c in args.command]
        lines += [""]
    return lines


def trace(args):
    rs = _rows(args.dirs[0], "kernel_trace.csv")
    disp = [(int(_col(r, "Dispatch_Id")), _col(r, "Kernel_Name")) for r in rs]
    start = _region_start(disp, args.first)
    agg = defaultdict(lambda: [0, 0.0])
    frames = 0
    for r in rs:
        i = int(_col(r, "Dispatch_Id"))
        name = _col(r, "Kernel_Name")
        if i < start or _is_copy(name) or "elementwise" in name:
            continue
        nm = f"{short(name)} | {_col(r, 'Grid_Size_X', 'Grid_Size')}"
        a = agg[nm]
        a[0] += 1
        a[1] += (int(_col(r, "End_Timestamp")) - int(_col(r, "Start_Timestamp"))) / 1e3
        if args.first != "__all__" and args.first in name:
            frames += 1
    total = sum(v[1] for v in agg.values())
    lines = _header(args, "Kernel trace")
    if frames:
        lines += [f"Profiled dispatches from id {start}; frames (dispatches of the marker kernel): {frames}.",
                  "Grid in threads.  us per frame = the kernel's total time / frames.", "",
                  "| kernel | grid | dispatches | mean us | us per frame | % of kernel time |",
                  "|---|---:|---:|---:|---:|---:|"]
    else:
        lines += ["Every dispatch of the run.  Grid in threads.", "",
                  "| kernel | grid | dispatches | mean us | total us | % of kernel time |",
                  "|---|---:|---:|---:|---:|---:|"]
    for k, (n, t) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        name, grid = k.split(" | ")
        col = t / frames if frames else t
        lines.append(f"| {name} | {grid} | {n} | {t / n:.2f} | {col:.2f} | {100 * t / total:.1f} |")
    return lines


def _pmc_table(d, marker):
    rs = _rows(d, "counter_collection.csv")
    disp = {}
    for r in rs:
        disp[int(_col(r, "Dispatch_Id"))] = _col(r, "Kernel_Name")
    start = _region_start(list(disp.items()), marker)
    agg = defaultdict(lambda: defaultdict(float))
    ids = defaultdict(set)
    copies = defaultdict(dict)
    for r in rs:
        i = int(_col(r, "Dispatch_Id"))
        name = _col(r, "Kernel_Name")
        c, v = _col(r, "Counter_Name"), float(_col(r, "Counter_Value"))
        if _is_copy(name):
            copies[i][c] = copies[i].get(c, 0.0) + v
            continue
        if i < start or "elementwise" in name:
            continue
        nm = f"{short(name)} | {_col(r, 'Grid_Size_X', 'Grid_Size')}"
        agg[nm][c] += v
        ids[nm].add(i)
    per = {k: {c: s / len(ids[k]) for c, s in v.items()} for k, v in agg.items()}
    count = {k: len(v) for k, v in ids.items()}
    # the calibration copy: the copy dispatch with the largest reading
    cal = {}
    for cv in copies.values():
        for c, v in cv.items():
            cal[c] = max(cal.get(c, 0.0), v)
    return start, per, count, cal


def pmc(args):
    start, per, count, _ = _pmc_table(args.dirs[0], args.first)
    counters = sorted({c for v in per.values() for c in v})
    lines = _header(args, "Counters")
    lines += [f"Profiled dispatches from id {start}.  Values per dispatch (mean over the dispatches).", "",
              "| kernel | grid | dispatches | " + " | ".join(counters) + " |",
              "|---|---:|---:|" + "---:|" * len(counters)]
    for k in sorted(per, key=lambda k: -max(per[k].values())):
        name, grid = k.split(" | ")
        lines.append(f"| {name} | {grid} | {count[k]} | " + " | ".join(f"{per[k].get(c, 0.0):.1f}" for c in counters)
                     + " |")
    return lines


def sources_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def hbm(args):
    _, fetch, nf, calf = _pmc_table(args.dirs[0], args.first)
    _, write, nw, calw = _pmc_table(args.dirs[1], args.first)
    kib = COPY_BYTES / 1024
    fscale = kib / calf["FETCH_SIZE"] if calf.get("FETCH_SIZE") else float("nan")
    wscale = kib / calw["WRITE_SIZE"] if calw.get("WRITE_SIZE") else float("nan")
    lines = _header(args, "HBM traffic")
    lines += ["FETCH_SIZE and WRITE_SIZE are KiB per dispatch, each from its own run.  Calibration: one plain",
              "256 MiB device-to-device copy in each run; scale = 262144 KiB / what the counter reads for it.", "",
              f"copy FETCH_SIZE: {calf.get('FETCH_SIZE', float('nan')):.1f} KiB -> fetch scale {fscale:.4f}",
              f"copy WRITE_SIZE: {calw.get('WRITE_SIZE', float('nan')):.1f} KiB -> write scale {wscale:.4f}", "",
              "| kernel | grid | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM MB per dispatch |",
              "|---|---:|---:|---:|---:|---:|"]
    for k in sorted(set(fetch) | set(write), key=lambda k: -fetch.get(k, {}).get("FETCH_SIZE", 0.0)):
        name, grid = k.split(" | ")
        f = fetch.get(k, {}).get("FETCH_SIZE", 0.0)
        w = write.get(k, {}).get("WRITE_SIZE", 0.0)
        mb = (f * fscale + w * wscale) * 1024 / 1e6
        lines.append(f"| {name} | {grid} | {nf.get(k, nw.get(k, 0))} | {f:.1f} | {w:.1f} | {mb:.2f} |")
    if args.sources:
        # machine-readable lines for the kernel named by --kernel (read by bench.py)
        key = next((k for k in fetch if k.split(" | ")[0] == args.kernel), None)
        if key is not None:
            f = fetch[key]["FETCH_SIZE"]
            w = write.get(key, {}).get("WRITE_SIZE", 0.0)
            lines += ["", f"kernel: {args.kernel}", f"dispatches: {nf[key]}",
                      f"fetch_size_kib_per_dispatch: {f:.1f}", f"write_size_kib_per_dispatch: {w:.1f}",
                      f"fetch_scale: {fscale:.4f}", f"write_scale: {wscale:.4f}",
                      f"hbm_bytes_per_launch: {(f * fscale + w * wscale) * 1024:.0f}",
                      f"kernel_sources_sha256: {sources_hash(args.sources)}",
                      "# kernel_sources_sha256: first 16 hex digits of sha256 over " + ", ".join(
                          os.path.basename(s) for s in args.sources) + " (in that order)"]
    return lines


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("mode", choices=["trace", "pmc", "hbm"])
    ap.add_argument("dirs", nargs="+")
    ap.add_argument("--first", default="blend_kernel")
    ap.add_argument("--title", default="")
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--sources", nargs="*", default=[])
    ap.add_argument("--kernel", default="blend_kernel<false>")
    ap.add_argument("--out", default="")
    args = ap.parse_args(argv)
    lines = {"trace": trace, "pmc": pmc, "hbm": hbm}[args.mode](args)
    text = "\n".join(lines) + "\n"
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(text)
    sys.stdout.write(text)


if __name__ == "__main__":
    main()
