"""Benchmark: RaRa-clipped frames per second on the general-scene workload
(1,000,000 Gaussians, SH degree 3, 1920x1080, 16 orbit views x 16 plane
offsets swept through the scene), scene resident in HBM, image left on the
device.  One step = one full frame (preprocess + bin/sort + render) for the
next (view, offset) of the sweep.

Prints one JSON line.  Besides the contract fields it reports the plain
(unclipped) frame rate over the same views, per-stage times from HIP events
on the launch stream, Gaussian-pixel evaluations per second, the roofline of
the dominant kernel and the FP64 oracle timed on a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RaRa-clipped FPS @1080p/1M Gaussians; served p50/p99 latency vs plain"

# Algorithmic work per Gaussian-pixel evaluation of the blend (FMA = 2 flops,
# exp/sqrt/reciprocal = 1): offset 2, quadratic form 8, exp and opacity 2,
# clamp and skip test 2, transmittance 3, colour 7  -> 24.
# CUTOFF extra: delta 9, D 3, P 3, P.D 5, D.D 5, s_m 2, closest point 6,
# |.|^2 5, h 3, near-root test 2, plane rate 4, midpoint value 4, weight 5 -> 56.
FLOPS_EVAL = 24
FLOPS_CUT = 56
PEAK_FP32 = 157.3e12          # MI355X FP32 vector, packed FMA
PEAK_FP32_UNPACKED = 78.6e12  # without packed FP32 (the kernels are compiled without it)
PEAK_HBM = 8.0e12

# frames in flight in the timed sweep (renderer.FramePipeline): one stream and
# one buffer set each
PIPE_STREAMS = 3


# rocprofv3 counter summary of the blend kernel on the general workload: HBM
# bytes per launch from FETCH_SIZE and WRITE_SIZE, scaled by what the same
# counters read for a plain device copy of known size.  Reported only while
# the blend's sources are the ones the counters were taken on.
COUNTER_FILE = os.path.join(ROOT, "profiles", "hbm_general_1080p.md")
# the blend's sources, and the header holding its schedule and batch constants
BLEND_SOURCES = ("paper_2506_20202_amd/csrc/blend.hip", "paper_2506_20202_amd/csrc/blend_common.h",
                 "paper_2506_20202_amd/csrc/rara_internal.h")


def blend_source_hash():
    h = hashlib.sha256()
    for f in BLEND_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def blend_traffic():
    try:
        with open(COUNTER_FILE) as fh:
            text = fh.read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if ":" in line and not line.startswith(("#", " ", "\t")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("kernel_sources_sha256") != blend_source_hash():
        return None
    return float(fields["hbm_bytes_per_launch"])


# rara_gaussians.sh_layout of the resident scenes: Gaussian-major [n][(D+1)^2][3]
# (a frame reads only the drawn Gaussians' coefficients) or coefficient-major
# [(D+1)^2][3][n]
SH_LAYOUTS = {"gaussian": 1, "coefficient": 0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=160)
    ap.add_argument("--reps", type=int, default=5, help="timed sweeps per variant; the median is reported")
    ap.add_argument("--no-secondary", action="store_true", help="skip the strand workload")
    ap.add_argument("--warmup", type=int, default=16)
    ap.add_argument("--workload", default="general", choices=["general", "strands", "multilayer", "box", "diff"],
                    help="headline workload (general); the others for profiler runs and secondary measurements")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-peaks", action="store_true", help="skip the copy and FMA-loop peak measurements")
    ap.add_argument("--serve-requests", type=int, default=2000, help="requests per load point")
    ap.add_argument("--serve-loads", type=float, nargs="+", default=[0.25, 0.5, 0.75, 0.9],
                    help="arrival rates as fractions of the saturation rate")
    ap.add_argument("--serve-budget-gib", type=float, default=32.0,
                    help="HBM for serving slots beyond the resident scenes")
    ap.add_argument("--serve-slots", type=int, default=64, help="slots kept (buffers and captured graphs)")
    ap.add_argument("--serve-inflight", type=int, default=8, help="frames running at once")
    ap.add_argument("--serve-lanes", type=int, default=3, help="streams (hardware queues) the frames run on")
    ap.add_argument("--sh-layout", default="coefficient", choices=sorted(SH_LAYOUTS),
                    help="layout of the resident scenes' SH coefficients (converted once at upload)")
    ap.add_argument("--profile-steps", type=int, default=0, help="only run this many frames (for profilers)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="with --profile-steps: also run one plain 256 MiB device copy at the end (counter "
                         "calibration)")
    return ap.parse_args()


def workload(name):
    """Scene, frame grid (grid[view][offset] = (camera, plane)) and description."""
    from paper_2506_20202_amd import scenes
    if name == "general":
        sc = scenes.general_scene(1)
        cams = scenes.general_views()
        planes = scenes.plane_sweep(sc, scenes.general_plane_normal(1), count=16)
        grid = [[(cams[v], planes[o]) for o in range(16)] for v in range(16)]
        desc = {"workload": "general scene, 1,000,000 Gaussians (64 clusters), SH3, 1920x1080, "
                            "16 orbit views x 16 plane offsets", "gaussians": sc.n, "width": 1920, "height": 1080,
                "views": 16, "plane_offsets": 16}
    elif name == "multilayer":
        return multilayer_workload()
    elif name == "box":
        return box_workload()
    else:
        sc = scenes.strand_scene(2)
        cams = scenes.strand_views()
        grid = [[(cams[v], p) for p in scenes.strand_planes(v)] for v in range(8)]
        desc = {"workload": "strand scene, 100,000 strands x 32 = 3,200,000 Gaussians, SH1, 1024x1024, "
                            "8 views x 4 oblique planes", "gaussians": sc.n, "width": 1024, "height": 1024,
                "views": 8, "plane_offsets": 4}
    return sc, grid, desc


def clip_order(clipping):
    """Order of the timed frames.  ``clipping[v]`` lists the plane offsets that
    clip in view v (Sec. 4.2's protocol sweeps a plane through the scene; a
    frame clips when the plane leaves some Gaussians CUTOFF and some
    INVISIBLE).  Frame i takes view v = i mod V and, with m = i div V, the
    offset clipping[v][(m + v) mod K_v]: every prefix strides views and
    offsets alike, and V * max(K_v) frames visit every clipping (view,
    offset) pair (each exactly once when all K_v are equal)."""
    V = len(clipping)
    if V == 0 or any(len(c) == 0 for c in clipping):
        raise ValueError("every view needs at least one clipping offset")
    K = max(len(c) for c in clipping)
    return [(i % V, clipping[i % V][(i // V + i % V) % len(clipping[i % V])]) for i in range(V * K)]


def count_evals(fr, n):
    """Work of the frame just rendered (measurement only): Gaussian-pixel
    evaluations by the method's definition (per pixel, the list entries up to
    termination, n_walked), the evaluations the blend kernel actually
    performed for live pixels (n_eval plane 0: entries its conservative
    quadrant / strip test lets reach the pixel), and the clip weights among
    those (n_eval plane 1)."""
    import torch
    walked = int(fr.out.n_walked.to(torch.int64).sum().item())
    ev = fr.out.n_eval.to(torch.int64).sum(dim=(1, 2)).cpu().tolist()
    return walked, int(ev[0]), int(ev[1])


def preprocess_bytes(n, sh_degree, live, drawn, cut_drawn):
    """Algorithmic HBM bytes of one preprocess launch: mean and scale (24 B),
    the label (1 B), tiles_touched (4 B) and the tile record (16 B: rectangle
    and listed-tile mask) of every Gaussian; the quaternion (16 B) of every
    Gaussian that is not INVISIBLE; opacity (4 B), SH coefficients
    (12 (D+1)^2 B) and the splat record and depth (52 B) of every drawn one;
    the 48 B ray record of a drawn CUTOFF one."""
    return 45 * n + 16 * live + (4 + 12 * (sh_degree + 1) ** 2 + 52) * drawn + 48 * cut_drawn


def bin_sort_bytes(n, drawn, pairs, tiles):
    """Algorithmic HBM bytes of rara_bin_sort as this sort runs it, each pass
    reading and writing its keys and values once: the first depth pass reads
    depth and tile count of every Gaussian and writes 8 B per drawn one, three
    more depth passes move 16 B per drawn Gaussian, the chunk sums read each
    drawn Gaussian's index and 16 B tile record and write the record in depth
    order (36 B), the emit reads index and record (20 B per drawn Gaussian) and
    writes 8 B per pair, the tile passes move 16 B per pair except the last,
    which writes only the values (12 B per pair), and the ranges and schedule
    take 12 B per tile."""
    tile_passes = max(1, (max(1, int(tiles - 1).bit_length()) + 7) // 8)
    return (8 * n + 8 * drawn + 48 * drawn + 56 * drawn + 8 * pairs + 16 * pairs * (tile_passes - 1) + 12 * pairs
            + 12 * tiles)


def _omp_threads(k=None):
    """Set (when k is given) and return the OpenMP thread count of the oracle."""
    import ctypes
    import oracle
    oracle.lib()
    gomp = ctypes.CDLL("libgomp.so.1")
    if k is not None:
        gomp.omp_set_num_threads(int(k))
    return int(gomp.omp_get_max_threads())


def oracle_frame(sc, cam, plane, budget_s):
    """The FP64 oracle on one frame: classify, project and sort in full, then
    composite evenly spaced tile rows within the time budget, scaled to the
    whole frame."""
    import oracle
    t0 = time.perf_counter()
    lab, dep, rad = oracle.classify(sc, plane)
    proj = oracle.project(sc, cam, lab)
    offs, ids = oracle.tile_lists(proj, cam)
    t_prep = time.perf_counter() - t0
    tx = (cam.width + 15) // 16
    rows = (cam.height + 15) // 16
    L = oracle.lib()

    def comp(t0_, t1_):
        W, H = cam.width, cam.height
        image = np.zeros((3, H, W)); fT = np.ones(H * W); nc = np.zeros(H * W, np.int32)
        nw = np.zeros(H * W, np.int32); fl = np.zeros(H * W, np.uint32); cnt = np.zeros(8, np.int64)
        bg = np.zeros(3, np.float32)
        pa = oracle.planes_of(plane)
        s = time.perf_counter()
        L.oracle_composite(sc.n, oracle._p(lab), oracle._p(proj["mean2d"]), oracle._p(proj["conic"]),
                           oracle._p(sc.opacity), oracle._p(proj["rgb"]), oracle._p(sc.mean), oracle._p(proj["minv"]),
                           oracle._p(pa), pa.shape[0], oracle.clip_mode(plane), oracle._p(oracle.cam_array(cam)), W,
                           H, oracle._p(bg), oracle._p(offs), oracle._p(ids), 3.0, 0, int(t0_), int(t1_), 1e-3,
                           oracle._p(image), oracle._p(fT), oracle._p(nc), oracle._p(nw), oracle._p(fl),
                           oracle._p(cnt))
        return time.perf_counter() - s, cnt
    mid = rows // 2
    t_row, _ = comp(mid * tx, (mid + 1) * tx)
    nrows = int(max(1, min(rows, (budget_s - t_prep) / max(t_row, 1e-6))))
    step = max(1, rows // nrows)
    picked = list(range(0, rows, step))[:nrows]
    t_comp, evals = 0.0, 0
    for r in picked:
        dt, cnt = comp(r * tx, (r + 1) * tx)
        t_comp += dt
        evals += int(cnt[0])
    frac = len(picked) / rows
    frame_s = t_prep + t_comp / frac
    return {"value": 1.0 / frame_s, "unit": "frames/s", "cores": _omp_threads(), "kind": "oracle",
            "sample": f"one {cam.width}x{cam.height} frame of {sc.n} Gaussians: classify/project/sort in full "
                      f"({t_prep:.2f} s), composite of {len(picked)} of {rows} tile rows ({t_comp:.2f} s) "
                      f"scaled to the frame",
            "geval_per_s": evals / t_comp / 1e9 if t_comp > 0 else None}


def cpu_baseline(general, strands, budget_s):
    """The oracle as it stands, on the host: the general 1080p frame (view 0,
    mid-sweep plane) on every core -- the reported value -- and on one core,
    plus the tiny frame and one strand frame on every core."""
    from paper_2506_20202_amd import scenes
    cores = _omp_threads()
    res = oracle_frame(*general, budget_s * 0.4)
    _omp_threads(1)
    res["single_core"] = oracle_frame(*general, budget_s * 0.3)
    _omp_threads(cores)
    tiny = scenes.tiny_scene(0)
    res["tiny"] = oracle_frame(tiny, scenes.tiny_camera(), scenes.tiny_plane(0), budget_s)
    if strands is not None:
        res["strands"] = oracle_frame(*strands, budget_s * 0.3)
    return res


def serve_bench(args):
    """Serving mix over multi-layer scenes: 3 resident scenes (5 shells of
    200k/300k/400k Gaussians, SH 0/2/3), requests with a random scene, a
    resolution from {512^2, 1024^2, 1920x1080, 2048^2}, a camera on a sphere of
    radius 5 and a random plane.  Saturation is measured from a burst; then
    Poisson arrivals at 0.25, 0.5, 0.75 and 0.9 of it, each the same request
    stream clipped and with clipping off (plain); then a run whose HBM budget
    leaves 1 GiB beyond the resident scenes, which forces queuing."""
    from paper_2506_20202_amd import scenes
    from paper_2506_20202_amd.serve import Engine
    rng = np.random.default_rng(3)
    defs = [("A", scenes.multilayer_scene(31, per_shell=200_000, sh_degree=0)),
            ("B", scenes.multilayer_scene(32, per_shell=300_000, sh_degree=2)),
            ("C", scenes.multilayer_scene(33, per_shell=400_000, sh_degree=3))]
    sizes = [(512, 512), (1024, 1024), (1920, 1080), (2048, 2048)]
    eng = Engine(hbm_budget=0, max_slots=args.serve_slots, max_inflight=args.serve_inflight, lanes=args.serve_lanes)
    for name, sc in defs:
        eng.add_scene(name, sc)
    resident = eng.ex.resident_bytes()
    graphs = eng.ex.use_graphs
    budget = resident + int(args.serve_budget_gib * (1 << 30))
    eng.sched.budget = budget

    def make(nreq):
        out = []
        for _ in range(nreq):
            name, sc = defs[int(rng.integers(3))]
            W, H = sizes[int(rng.integers(4))]
            out.append((name, scenes.random_camera_on_sphere(rng, 5.0, W, H), scenes.random_plane_through(rng, sc)))
        return out

    # warm-up: every shape class once (slots built)
    for name, _ in defs:
        for W, H in sizes:
            eng.submit(name, scenes.random_camera_on_sphere(rng, 5.0, W, H), scenes.random_plane_through(rng, defs[0][1]))
    eng.run_until_idle()
    # saturation: a burst of requests all queued at once
    burst = make(128)
    t0 = time.perf_counter()
    for r in burst:
        eng.submit(*r)
    eng.run_until_idle()
    sat = len(burst) / (time.perf_counter() - t0)

    def run(reqs, gaps, clipped):
        eng.sched.latencies.clear()
        eng.sched.completed.clear()
        eng.ex.batches.clear()
        eng.sched.max_inflight = 0
        ev0 = eng.sched.evictions
        # every request is submitted up front with its Poisson arrival time; the
        # scheduler admits it once that time has come (no host thread spins)
        t_start = time.perf_counter() + 0.05
        t = t_start
        futs = []
        for (name, cam, pl), gap in zip(reqs, gaps):
            t += gap
            p = pl if clipped else type(pl)(pl.n, pl.d, False)
            futs.append(eng.submit(name, cam, p, arrival=t))
        eng.start()
        for f in futs:
            f.result(timeout=600)
        wall = time.perf_counter() - t_start
        eng.stop()
        st = eng.stats()
        mpix = sum(c.width * c.height for _, c, _ in reqs) / 1e6
        return {"p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "mean_ms": st["mean_ms"],
                "throughput_req_s": len(reqs) / wall, "throughput_mpix_s": mpix / wall,
                "max_inflight": st["max_inflight"], "retries": st["retries"],
                "evictions": eng.sched.evictions - ev0, "mean_batch": st.get("mean_batch"),
                "max_batch": st.get("max_batch")}

    loads = []
    for frac in args.serve_loads:
        rate = frac * sat
        reqs = make(args.serve_requests)
        gaps = rng.exponential(1.0 / rate, len(reqs))
        clipped = run(reqs, gaps, True)
        plain = run(reqs, gaps, False)
        loads.append({"load_fraction": frac, "offered_req_s": rate, "requests": len(reqs), "clipped": clipped,
                      "plain": plain})
        print(f"[bench] serving at {frac:.2f} x saturation ({rate:.0f} req/s): clipped p50 {clipped['p50_ms']:.2f} "
              f"p99 {clipped['p99_ms']:.2f} ms, plain p50 {plain['p50_ms']:.2f} p99 {plain['p99_ms']:.2f} ms",
              file=sys.stderr, flush=True)
    # a tight HBM budget: resident scenes plus 1 GiB of slots, so requests queue for memory
    for sl in list(eng.sched.slots):
        if sl.request is None:
            eng.sched._drop(sl)
    eng.sched.budget = resident + (1 << 30)
    reqs = make(max(200, args.serve_requests // 4))
    rate = 0.5 * sat
    gaps = rng.exponential(1.0 / rate, len(reqs))
    tight = dict(run(reqs, gaps, True), hbm_budget_gib=eng.sched.budget / 2 ** 30, offered_req_s=rate,
                 requests=len(reqs), load_fraction=0.5)
    print(f"[bench] serving with 1 GiB of slots: p50 {tight['p50_ms']:.2f} p99 {tight['p99_ms']:.2f} ms, "
          f"{tight['evictions']} evictions", file=sys.stderr, flush=True)
    eng.close()
    return {"workload": "3 resident multi-layer scenes (1.0M SH0, 1.5M SH2, 2.0M SH3), resolutions "
                        "512^2/1024^2/1920x1080/2048^2, camera on a radius-5 sphere, random plane",
            "saturation_req_s": sat, "hbm_budget_gib": budget / 2 ** 30, "max_slots": args.serve_slots,
            "max_inflight": args.serve_inflight, "lanes": args.serve_lanes, "graphs": graphs,
            "batched_blends": eng.ex.batch, "loads": loads, "tight_budget": tight}


def measured_peaks(reps: int = 5):
    """Attainable peaks on this GPU (libpeak.so): a streaming copy of 1 GiB
    (larger than the 256 MB Infinity Cache) and 8192 workgroups of
    independent unpacked FP32 FMA chains, each the best of ``reps`` runs timed
    with HIP events on the launch stream."""
    import torch
    from paper_2506_20202_amd import binding as B
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    sp = int(stream.cuda_stream)
    nbytes = 1 << 30
    src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    out = torch.zeros(8192 * 256, dtype=torch.float32, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def best(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) / 1e3)
        return min(ts)

    t_copy = best(lambda: B.peak_copy(dst.data_ptr(), src.data_ptr(), nbytes, 256 * 32, sp))
    flops = [0.0]

    def fma():
        flops[0] = B.peak_fma(out.data_ptr(), 8192, 4096, sp)
    t_fma = best(fma)
    res = {"hbm_copy_gbs": 2 * nbytes / t_copy / 1e9, "hbm_copy_bytes": 2 * nbytes,
           "fp32_fma_tflops": flops[0] / t_fma / 1e12,
           "copy_frac_of_spec": 2 * nbytes / t_copy / PEAK_HBM,
           "fma_frac_of_unpacked_spec": flops[0] / t_fma / PEAK_FP32_UNPACKED,
           "note": "copy: 1 GiB read + 1 GiB written; FMA: unpacked v_fma_f32, 16 independent chains per lane"}
    del src, dst, out
    torch.cuda.empty_cache()
    print(f"[bench] measured peaks: copy {res['hbm_copy_gbs']:.0f} GB/s, FMA {res['fp32_fma_tflops']:.1f} TFLOP/s",
          file=sys.stderr, flush=True)
    return res


def profile_run(args, sc, grid, dev):
    """Profiler runs (rocprofv3): preprocess + bin_sort over every frame of the
    grid (capacity and labels, no blend; the initial capacity of 8 pairs per
    Gaussian holds every frame of the workloads here, so each of those kernels
    runs once per grid frame), then warmup + profile_steps whole frames in the
    timed order over the frames that clip, as in the timed run: each kernel's
    last warmup + profile_steps dispatches are those frames."""
    import torch
    from paper_2506_20202_amd import renderer as R
    ds = R.DeviceScene.from_scene(sc, dev, sh_layout=SH_LAYOUTS[args.sh_layout])
    W, H = grid[0][0][0].width, grid[0][0][0].height
    fr = R.Frame(sc.n, W, H, 8 * sc.n, dev, walked=False, pair_start=False, sorted_keys=False)
    cap0 = fr.capacity
    maxP, _, order = scan_grid(ds, fr, grid)
    fr.grow(int(maxP * 1.05) + 4096)
    torch.cuda.synchronize()
    for i in range(args.warmup + args.profile_steps):
        v, o = order[i % len(order)]
        R.enqueue_frame(ds, fr, *grid[v][o])
    torch.cuda.synchronize()
    assert int(fr.bins.overflow.item()) == 0
    if args.calibrate_copy:
        calibration_copy(dev)
    print(json.dumps({"profile_steps": args.profile_steps, "warmup": args.warmup, "pair_capacity": fr.capacity,
                      "scan_capacity": cap0, "scan_grew": maxP > cap0, "grid_frames": len(grid) * len(grid[0]),
                      "frames": [list(order[i % len(order)]) for i in range(args.warmup + args.profile_steps)],
                      "copy_bytes": (256 << 20) if args.calibrate_copy else 0}))


def calibration_copy(dev):
    """One plain 256 MiB device-to-device copy, whose FETCH_SIZE and
    WRITE_SIZE readings scale the other kernels' (rocprofv3 --pmc runs)."""
    import torch
    src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def scan_grid(ds, fr, grid):
    """Preprocess + bin_sort of every frame of the grid (no blend; the pair
    capacity of ``fr`` grows as needed): the largest pair count, the label
    counts of each (view, offset) from the device's labels, and the timed
    order over the frames that clip (``clip_order``)."""
    import torch
    from paper_2506_20202_amd import renderer as R
    n = ds.n
    maxP, labels = 0, {}
    for v, row in enumerate(grid):
        for o, (cam, pl) in enumerate(row):
            R.enqueue_frame(ds, fr, cam, pl, stages=("pre", "bin"))
            torch.cuda.synchronize()
            P = int(fr.bins.num_pairs.item())
            if int(fr.bins.overflow.item()):
                fr.grow(max(int(P * 1.25) + 1024, fr.capacity * 2))
                R.enqueue_frame(ds, fr, cam, pl, stages=("pre", "bin"))
                torch.cuda.synchronize()
                assert not int(fr.bins.overflow.item())
            maxP = max(maxP, P)
            cnt = torch.bincount(fr.proj.label[:n].to(torch.int64), minlength=3).cpu().tolist()
            labels[(v, o)] = {"visible": cnt[1], "cutoff": cnt[2], "invisible": cnt[0]}
    clipping = [[o for o in range(len(row)) if labels[(v, o)]["cutoff"] > 0 and labels[(v, o)]["invisible"] > 0]
                for v, row in enumerate(grid)]
    return maxP, labels, clip_order(clipping)


def measure(sc, grid, args, reps, label):
    """Frames per second with clipping (RaRa), without a plane (Original) and
    with hard clipping (Hard), over the frames of ``grid`` that clip, in the
    order of ``clip_order``: each the median of ``reps`` timed sweeps of
    args.steps frames, rendered two ways: one frame after the other on one
    stream ("serial"), and with PIPE_STREAMS frames in flight
    (renderer.FramePipeline: consecutive frames on their own streams overlap).
    The whole grid, non-clipping frames included, is timed too.  Per-stage
    times and work counts over exactly the timed frames."""
    import torch
    from paper_2506_20202_amd import renderer as R
    dev = torch.device("cuda:0")
    ds = R.DeviceScene.from_scene(sc, dev, sh_layout=SH_LAYOUTS[args.sh_layout])
    V, O = len(grid), len(grid[0])
    W, H = grid[0][0][0].width, grid[0][0][0].height
    stream = torch.cuda.current_stream(dev)
    # capacity and labels from one pass over every frame (outside the timed region)
    fr = R.Frame(sc.n, W, H, 8 * sc.n, dev, walked=False, pair_start=False, sorted_keys=False)
    maxP, labels, order = scan_grid(ds, fr, grid)
    frames = [grid[v][o] for v, o in order]
    sweep = [grid[v][o] for o in range(O) for v in range(V)]
    variants = {"rara": frames,
                "original": [(cam, dataclasses.replace(pl, enabled=0)) for cam, pl in frames],
                "hard": [(cam, dataclasses.replace(pl, enabled=2)) for cam, pl in frames]}
    if args.no_plain:
        del variants["original"], variants["hard"]
    for name, fl in variants.items():
        if name != "rara":
            for cam, pl in fl[:: max(1, len(fl) // 16)]:
                R.render_checked(ds, fr, cam, pl)
                maxP = max(maxP, int(fr.bins.num_pairs.item()))
    fr.grow(int(maxP * 1.05) + 4096)
    pipe = R.FramePipeline(ds, W, H, fr.capacity, streams=PIPE_STREAMS, walked=False)
    torch.cuda.synchronize()
    print(f"[bench] {label}: max pairs {maxP}, capacity {fr.capacity}, {len(order)} clipping frames "
          f"of {V * O}", file=sys.stderr, flush=True)

    def run_serial(frame_list, k):
        for i in range(k):
            cam, pl = frame_list[i % len(frame_list)]
            R.enqueue_frame(ds, fr, cam, pl)

    def run_pipe(frame_list, k):
        pipe.start(stream)
        for i in range(k):
            cam, pl = frame_list[i % len(frame_list)]
            pipe.submit(cam, pl)
        pipe.join(stream)

    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(run, fl, check, steps):
        run(fl, args.warmup)
        torch.cuda.synchronize()
        vals = []
        for _ in range(reps):
            torch.cuda.synchronize()
            ev0.record(stream)
            run(fl, steps)
            ev1.record(stream)
            torch.cuda.synchronize()
            vals.append(steps / (ev0.elapsed_time(ev1) / 1e3))
            assert not check()
        return {"median": float(np.median(vals)), "reps": vals}

    fps, fps_serial = {}, {}
    for name, fl in variants.items():
        fps_serial[name] = timed(run_serial, fl, lambda: int(fr.bins.overflow.item()), args.steps)
        fps[name] = timed(run_pipe, fl, pipe.overflowed, args.steps)
        print(f"[bench] {label} {name}: {fps[name]['median']:.1f} FPS pipelined, "
              f"{fps_serial[name]['median']:.1f} serial (medians of {reps})", file=sys.stderr, flush=True)
    # the whole grid in sweep order, frames that clip nothing included
    full_sweep = {"pipelined": timed(run_pipe, sweep, pipe.overflowed, len(sweep))["median"],
                  "serial": timed(run_serial, sweep, lambda: int(fr.bins.overflow.item()), len(sweep))["median"],
                  "frames": len(sweep)}
    pipe.close()
    del pipe

    # per-stage times (HIP events on the launch stream) and work counts over
    # the timed frames; each stage is timed over kRepeat back-to-back runs on
    # the same inputs (each run rewrites the same outputs), so its figure is
    # the kernels' own duration rather than that of an isolated launch.  The
    # work counts come from one more render into images with the n_walked
    # output, untimed.
    kRepeat = 4
    frw = R.Frame(sc.n, W, H, 1, dev, walked=True)
    frw.proj, frw.bins = fr.proj, fr.bins
    stage_ms = {"preprocess": 0.0, "bin_sort": 0.0, "render": 0.0}
    E_tot, Ev_tot, Ecut_tot, P_tot, n_live, n_drawn, n_cut_drawn = 0, 0, 0, 0, 0, 0, 0
    bytes_pre, bytes_bin = 0, 0
    nst = args.steps
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    for i in range(nst):
        cam, pl = frames[i % len(frames)]
        evs[0].record(stream)
        for _ in range(kRepeat):
            R.enqueue_frame(ds, fr, cam, pl, stages=("pre",))
        evs[1].record(stream)
        for _ in range(kRepeat):
            R.enqueue_frame(ds, fr, cam, pl, stages=("bin",))
        evs[2].record(stream)
        for _ in range(kRepeat):
            R.enqueue_frame(ds, fr, cam, pl, stages=("render",))
        evs[3].record(stream)
        R.enqueue_frame(ds, frw, cam, pl, stages=("render",))
        torch.cuda.synchronize()
        stage_ms["preprocess"] += evs[0].elapsed_time(evs[1]) / kRepeat
        stage_ms["bin_sort"] += evs[1].elapsed_time(evs[2]) / kRepeat
        stage_ms["render"] += evs[2].elapsed_time(evs[3]) / kRepeat
        E, Ev, Ec = count_evals(frw, sc.n)
        E_tot += E
        Ev_tot += Ev
        Ecut_tot += Ec
        P_tot += int(fr.bins.num_pairs.item())
        lab = fr.proj.label[: sc.n]
        drawn = fr.proj.tiles_touched[: sc.n] != 0
        n_live += int((lab != 0).sum().item())
        n_drawn += int(drawn.sum().item())
        n_cut_drawn += int((drawn & (lab == 2)).sum().item())
        live_i, drawn_i = int((lab != 0).sum().item()), int(drawn.sum().item())
        bytes_pre += preprocess_bytes(sc.n, sc.sh_degree, live_i, drawn_i, int((drawn & (lab == 2)).sum().item()))
        bytes_bin += bin_sort_bytes(sc.n, drawn_i, int(fr.bins.num_pairs.item()), ((W + 15) // 16) * ((H + 15) // 16))
    for k in stage_ms:
        stage_ms[k] /= nst
    render_s = stage_ms["render"] / 1e3
    flops = (Ev_tot * FLOPS_EVAL + Ecut_tot * FLOPS_CUT) / nst
    timed_pairs = sorted(set(order[i % len(order)] for i in range(nst)))
    out = {"fps": fps, "fps_serial": fps_serial, "full_sweep": full_sweep, "stage_ms": stage_ms,
           "pairs_per_frame": P_tot / nst, "live_gaussians_per_frame": n_live / nst,
           "drawn_gaussians_per_frame": n_drawn / nst, "cutoff_drawn_per_frame": n_cut_drawn / nst,
           "evals_per_frame": E_tot / nst, "evaluated_per_frame": Ev_tot / nst,
           "cutoff_weights_per_frame": Ecut_tot / nst,
           "geval_per_s": E_tot / nst / render_s / 1e9, "flops_per_launch": flops,
           "blend_tflops": flops / render_s / 1e12, "pair_capacity": fr.capacity,
           "preprocess_bytes_per_launch": bytes_pre / nst, "bin_sort_bytes_per_frame": bytes_bin / nst,
           "timed_frames": [[v, o, labels[(v, o)]["cutoff"], labels[(v, o)]["invisible"]] for v, o in timed_pairs],
           "timed_order_head": [list(order[i % len(order)]) for i in range(min(nst, 32))],
           "clipping_frames": len(order), "grid_frames": V * O,
           "labels_by_offset_view0": [[labels[(0, o)]["visible"], labels[(0, o)]["cutoff"],
                                       labels[(0, o)]["invisible"]] for o in range(O)]}
    del fr, frw, ds
    torch.cuda.empty_cache()
    return out


def multilayer_workload():
    """One of the serving scenes (5 nested shells, 1.5M Gaussians, SH2) at
    1024x1024: 8 cameras on a radius-5 sphere x 4 planes through the scene."""
    from paper_2506_20202_amd import scenes
    rng = np.random.default_rng(8)
    sc = scenes.multilayer_scene(32, per_shell=300_000, sh_degree=2)
    cams = [scenes.random_camera_on_sphere(rng, 5.0, 1024, 1024) for _ in range(8)]
    planes = [scenes.random_plane_through(rng, sc) for _ in range(4)]
    grid = [[(c, p) for p in planes] for c in cams]
    desc = {"workload": "multi-layer scene, 5 shells x 300,000 = 1,500,000 Gaussians, SH2, 1024x1024, "
                        "8 cameras x 4 planes", "gaussians": sc.n, "width": 1024, "height": 1024}
    return sc, grid, desc


def box_workload():
    """Box clipping of a layered field, the case the paper cites for clip
    regions: the 1.5M-Gaussian multi-layer scene at 1024x1024, 8 cameras on a
    radius-5 sphere x 8 axis-aligned boxes (six half-spaces each) around a
    point near the centre, from one holding every shell to one inside the
    innermost."""
    from paper_2506_20202_amd import scenes
    rng = np.random.default_rng(9)
    sc = scenes.multilayer_scene(32, per_shell=300_000, sh_degree=2)
    cams = [scenes.random_camera_on_sphere(rng, 5.0, 1024, 1024) for _ in range(8)]
    c = rng.uniform(-0.2, 0.2, 3)
    boxes = [scenes.box_region(c - h * np.array([1.0, 0.8, 0.9]), c + h * np.array([0.9, 1.0, 0.8]))
             for h in np.linspace(2.3, 0.5, 8)]
    grid = [[(cam, b) for b in boxes] for cam in cams]
    desc = {"workload": "box clipping: multi-layer scene, 1,500,000 Gaussians, SH2, 1024x1024, 8 cameras x 8 "
                        "boxes (half-sizes 2.3 to 0.5 around a point near the centre)",
            "gaussians": sc.n, "width": 1024, "height": 1024}
    return sc, grid, desc


def backward_bytes(n, D, drawn, cut, pairs, pixels):
    """Algorithmic HBM bytes of one rara_render_backward: per pixel final_T,
    n_contrib and dL/dimage (20 B); per pair its list entry (4 B) and its
    84-byte gradient slot written once and read once; per drawn Gaussian its
    splat record (48 B, and the 48-byte ray record of a CUTOFF one) and its
    84-byte slot sum written and read; per Gaussian the raw parameters read
    and their gradients written (44 + 12 (D+1)^2 B each way)."""
    per_g = 44 + 12 * (D + 1) ** 2
    return 20 * pixels + pairs * (4 + 2 * 84) + drawn * (48 + 2 * 84) + 48 * cut + 2 * per_g * n


def backward_roofline(sc, cam, plane, fr, params, target, p4, reps):
    """One view's rara_render_backward through the C ABI, timed with HIP
    events on the stream it runs on (median of ``reps``), against its
    algorithmic bytes (backward_bytes)."""
    import torch
    from paper_2506_20202_amd import autograd as AG
    from paper_2506_20202_amd import binding as B
    dev = params[0].device
    with torch.no_grad():
        img = AG.render(*params, p4(plane), cam, True, frame=fr)
        dimg = (2.0 * (img - target) / img.numel()).contiguous()
    g = [torch.empty_like(p) for p in params]
    dplane = torch.empty(4, dtype=torch.float32, device=dev)
    gs = B.Grads()
    gs.mean, gs.scale, gs.quat, gs.opacity, gs.sh = (x.data_ptr() for x in g)
    gs.plane = dplane.data_ptr()
    ws_bytes = B.workspace_bytes(B.RARA_WS_BACKWARD, sc.n, fr.capacity, fr.width, fr.height)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    from paper_2506_20202_amd import renderer as R
    ds = R.DeviceScene(*(p.detach() for p in params), sc.sh_degree)
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    pl = rara_plane_of(plane)
    ms = []
    for _ in range(reps + 1):
        e0.record(stream)
        B.render_backward(ds.struct(), B.make_camera(cam), B.make_plane(pl), (0.0, 0.0, 0.0), fr.proj.struct(),
                          fr.bins.struct(), fr.capacity, fr.out.final_T.data_ptr(), fr.out.n_contrib.data_ptr(),
                          dimg.data_ptr(), gs, ws.data_ptr(), ws_bytes, int(stream.cuda_stream))
        e1.record(stream)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    ms = float(np.median(ms[1:]))
    lab = fr.proj.label[: sc.n]
    drawn = fr.proj.tiles_touched[: sc.n] != 0
    nd, ncut = int(drawn.sum().item()), int((drawn & (lab == 2)).sum().item())
    P = int(fr.bins.num_pairs.item())
    by = backward_bytes(sc.n, sc.sh_degree, nd, ncut, P, cam.width * cam.height)
    gbs = by / (ms / 1e3) / 1e9
    return {"kernel": "rara_render_backward of one view (blend_backward, slot_sum, project_backward, "
                      "plane_finalize)", "bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s",
            "frac": gbs / 8000.0, "bytes_per_launch": by, "avg_launch_ms": ms, "pairs": P, "drawn": nd,
            "note": "the blend_backward walk dominates and is latency-bound, far from this bound"}


def rara_plane_of(plane):
    """The plane as the forward's autograd path builds it (clip mode 1)."""
    from paper_2506_20202_amd.scenes import Plane
    return Plane(np.asarray(plane.n, np.float32), float(plane.d), 1)


def diff_bench(reps):
    """The differentiable workload: 500k general-scene Gaussians (SH3), 8 views
    at 800x800, each with its own clip plane, mean L2 loss against targets
    rendered from a perturbed copy.  One batch = 8 forwards + the backward of
    the loss; the forwards alone are timed too.  Median of `reps` batches."""
    import torch
    from paper_2506_20202_amd import autograd as AG
    from paper_2506_20202_amd import renderer as R
    from paper_2506_20202_amd import scenes
    dev = torch.device("cuda:0")
    sc = scenes.general_scene(4, n=500_000)
    cams, planes = scenes.diff_views(scene=sc)
    tgt = scenes.perturbed(sc)
    frames = [R.Frame(sc.n, c.width, c.height, 16 * sc.n, dev, walked=False, sorted_keys=False) for c in cams]

    def t(a, g=True):
        return torch.tensor(np.asarray(a), dtype=torch.float32, device=dev, requires_grad=g)

    def p4(pl, g=False):
        return torch.tensor([float(pl.n[0]), float(pl.n[1]), float(pl.n[2]), float(pl.d)], requires_grad=g)

    with torch.no_grad():
        tp = [t(a, False) for a in (tgt.mean, tgt.scale, tgt.quat, tgt.opacity, tgt.sh)]
        targets = [AG.render(*tp, p4(pl), cam, True, frame=fr) for cam, pl, fr in zip(cams, planes, frames)]
    params = [t(a) for a in (sc.mean, sc.scale, sc.quat, sc.opacity, sc.sh)]

    def forward():
        loss = 0.0
        for cam, pl, fr, tg in zip(cams, planes, frames, targets):
            img = AG.render(*params, p4(pl, True), cam, True, frame=fr, check=False)
            loss = loss + ((img - tg) ** 2).mean()
        return loss / len(cams)

    def checked():
        # the views' overflow flags, read once per batch
        if AG.overflowed(frames):
            raise RuntimeError("a view of the differentiable batch overflowed its pair capacity")

    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream(dev)

    def timed(fn):
        torch.cuda.synchronize()
        ev0.record(stream)
        fn()
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1)

    def batch():
        for p in params:
            p.grad = None
        forward().backward()
        checked()

    def fwd_only():
        with torch.no_grad():
            forward()
        checked()

    batch()
    fwd_only()
    b = [timed(batch) for _ in range(reps)]
    f = [timed(fwd_only) for _ in range(reps)]
    ok = all(bool(torch.isfinite(p.grad).all()) for p in params)
    roof = backward_roofline(sc, cams[0], planes[0], frames[0], params, targets[0], p4, reps)
    out = {"workload": "500,000 general-scene Gaussians, SH3, 8 views x 800x800, one clip plane per view, "
                       "L2 loss against a perturbed-scene target", "batch_ms": float(np.median(b)),
           "forward_ms": float(np.median(f)), "backward_ms": float(np.median(b) - np.median(f)),
           "reps": reps, "gradients_finite": ok, "roofline": roof,
           "note": "the views' pair-capacity overflow flags are read once per batch (one synchronisation)"}
    del frames, params, targets
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: there is no multi-GPU path (asked for --gpus {args.gpus}); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2506_20202_amd import renderer as R

    dev = torch.device("cuda:0")
    t_setup = time.perf_counter()
    if args.workload == "diff":
        if not args.profile_steps:
            sys.exit("--workload diff is a profiler run: give --profile-steps")
        print(json.dumps(diff_bench(args.profile_steps)))
        if args.calibrate_copy:
            calibration_copy(dev)
        return
    sc, grid, desc = workload(args.workload)
    print(f"[bench] scene n={sc.n} ready in {time.perf_counter() - t_setup:.1f}s", file=sys.stderr, flush=True)

    if args.profile_steps:
        profile_run(args, sc, grid, dev)
        return

    main_m = measure(sc, grid, args, args.reps, args.workload)
    fps = main_m["fps"]["rara"]["median"]
    ms_per_step = 1e3 / fps
    st = main_m["stage_ms"]
    pre_gbs = main_m["preprocess_bytes_per_launch"] / (st["preprocess"] / 1e3) / 1e9
    bin_gbs = main_m["bin_sort_bytes_per_frame"] / (st["bin_sort"] / 1e3) / 1e9
    roofline = {"bound": "alu", "kernel": "blend_kernel (rara_render)", "achieved": main_m["blend_tflops"],
                "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s", "frac": main_m["blend_tflops"] * 1e12 / PEAK_FP32,
                "traffic": blend_traffic(), "flops_per_launch": main_m["flops_per_launch"],
                "evaluated_per_launch": main_m["evaluated_per_frame"],
                "cutoff_weights_per_launch": main_m["cutoff_weights_per_frame"],
                "walked_evals_per_launch": main_m["evals_per_frame"],
                "flops_model": f"{FLOPS_EVAL} per evaluation the kernel performs for a live pixel + {FLOPS_CUT} per "
                               "clip weight it evaluates (FMA = 2, exp/rcp/sqrt = 1)",
                "avg_launch_ms": st["render"],
                "frac_of_unpacked_fp32": main_m["blend_tflops"] * 1e12 / PEAK_FP32_UNPACKED,
                "window": "the timed frames (every frame clips)",
                "stages": {
                    "preprocess": {"bound": "hbm", "unit": "GB/s", "achieved": pre_gbs, "peak": PEAK_HBM / 1e9,
                                   "frac": pre_gbs * 1e9 / PEAK_HBM,
                                   "bytes_per_launch": main_m["preprocess_bytes_per_launch"],
                                   "avg_launch_ms": st["preprocess"]},
                    "bin_sort": {"bound": "hbm", "unit": "GB/s", "achieved": bin_gbs, "peak": PEAK_HBM / 1e9,
                                 "frac": bin_gbs * 1e9 / PEAK_HBM,
                                 "bytes_per_frame": main_m["bin_sort_bytes_per_frame"],
                                 "avg_frame_ms": st["bin_sort"], "note": "all kernels of rara_bin_sort, from the "
                                 "first launch's start to the last one's end"}}}
    peaks = measured_peaks() if not args.no_peaks else None
    if peaks:
        roofline["frac_of_measured_fp32"] = main_m["blend_tflops"] / peaks["fp32_fma_tflops"]
        roofline["stages"]["preprocess"]["frac_of_measured_copy"] = pre_gbs / peaks["hbm_copy_gbs"]
        roofline["stages"]["bin_sort"]["frac_of_measured_copy"] = bin_gbs / peaks["hbm_copy_gbs"]

    secondary = {}
    strand_case = None
    if args.workload == "general" and not args.no_secondary:
        ssc, sgrid, sdesc = workload("strands")
        sm = measure(ssc, sgrid, args, max(1, args.reps // 2), "strands")
        secondary["strands"] = dict(sdesc, **sm)
        strand_case = (ssc, *sgrid[0][1])
        msc, mframes, mdesc = multilayer_workload()
        mm = measure(msc, mframes, args, max(1, args.reps // 2), "multilayer")
        secondary["multilayer"] = dict(mdesc, **mm)
        del msc, mframes
        bsc, bframes, bdesc = box_workload()
        bm = measure(bsc, bframes, args, max(1, args.reps // 2), "box")
        secondary["box"] = dict(bdesc, **bm)
        del bsc, bframes
        secondary["differentiable"] = diff_bench(3)
        print(f"[bench] differentiable batch {secondary['differentiable']['batch_ms']:.2f} ms "
              f"(forward {secondary['differentiable']['forward_ms']:.2f} ms)", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        gcase = (sc, *grid[0][8]) if args.workload == "general" else (sc, *grid[0][1])
        cpu = cpu_baseline(gcase, strand_case, args.cpu_seconds)
        print(f"[bench] oracle: {cpu['value']:.4f} frames/s on {cpu['cores']} threads, "
              f"{cpu['single_core']['value']:.4f} on 1", file=sys.stderr, flush=True)

    serving = None
    if not args.no_serve:
        serving = serve_bench(args)
        print(f"[bench] serving: saturation {serving['saturation_req_s']:.0f} req/s", file=sys.stderr, flush=True)

    plain = main_m["fps"].get("original", {}).get("median")
    hard = main_m["fps"].get("hard", {}).get("median")
    out = {
        "metric": METRIC, "value": fps, "unit": "frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": dict(desc, parallelism="single GPU", pair_capacity=main_m["pair_capacity"],
                       sh_layout=("Gaussian-major [n][(D+1)^2][3], converted once when the scene is uploaded"
                                  if args.sh_layout == "gaussian" else "coefficient-major [(D+1)^2][3][n]"),
                       timing=f"median of {args.reps} sweeps of {args.steps} frames, {PIPE_STREAMS} in flight "
                              "(frame i on stream i mod 3); the frames are the (view, offset) pairs whose plane "
                              "leaves Gaussians both CUTOFF and INVISIBLE, frame i taking view i mod V and "
                              "the ((i div V + i mod V) mod K)-th such offset",
                       clipping_frames=main_m["clipping_frames"], grid_frames=main_m["grid_frames"],
                       timed_frames_view_offset_cutoff_invisible=main_m["timed_frames"],
                       timed_order_head=main_m["timed_order_head"],
                       labels_by_offset_view0_visible_cutoff_invisible=main_m["labels_by_offset_view0"]),
        "plain_fps": plain, "hard_fps": hard, "clipped_over_plain_frame_time": (plain / fps) if plain else None,
        "rara_over_hard_frame_time": (hard / fps) if hard else None,
        "table1_protocol": {"original_fps": plain, "hard_fps": hard, "rara_fps": fps,
                            "frames": "the timed clipping frames"},
        "full_sweep": main_m["full_sweep"],
        "fps_reps": main_m["fps"]["rara"]["reps"],
        "serial": {k: v["median"] for k, v in main_m["fps_serial"].items()},
        "serial_ms_per_frame": 1e3 / main_m["fps_serial"]["rara"]["median"],
        "stage_ms": main_m["stage_ms"], "pairs_per_frame": main_m["pairs_per_frame"],
        "live_gaussians_per_frame": main_m["live_gaussians_per_frame"],
        "drawn_gaussians_per_frame": main_m["drawn_gaussians_per_frame"], "geval_per_s": main_m["geval_per_s"],
        "roofline": roofline, "measured_peaks": peaks, "cpu_baseline": cpu, "serving": serving,
        "secondary": secondary or None,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
