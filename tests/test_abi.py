"""CPU tests of the C ABI: the library loads, exports every function the
header declares, and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rara.h")


@pytest.fixture(scope="module")
def B():
    from paper_2506_20202_amd import binding, build
    if not os.path.exists(binding.LIB_PATH):
        build.build()
    return binding


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rara_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("rara_preprocess", "rara_bin_sort", "rara_render", "rara_render_backward", "rara_workspace_bytes",
              "rara_status_string"):
        assert f in names


def test_library_exports_every_declared_symbol(B):
    lib = B.lib()
    nm = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\s[TW]\s+(\S+)", nm))
    for f in declared_functions():
        assert f in exported, f
        assert hasattr(lib, f)
    assert set(B.EXPORTS) <= set(declared_functions())


def test_peak_library_exports_its_header(B):
    """libpeak.so (include/rara_peak.h), the attainable-peak probes the
    benchmark measures its roofline fractions against, loads and exports every
    function its header declares; bad arguments are refused without a launch."""
    hdr = open(os.path.join(ROOT, "include", "rara_peak.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    declared = sorted(set(re.findall(r"\b(rara_peak_[a-z_]+)\s*\(", hdr)))
    assert declared == sorted(B.PEAK_EXPORTS)
    L = B.peak_lib()
    nm = subprocess.run(["nm", "-D", "--defined-only", B.PEAK_LIB_PATH], capture_output=True, text=True,
                        check=True).stdout
    exported = set(re.findall(r"\s[TW]\s+(\S+)", nm))
    for f in declared:
        assert f in exported and hasattr(L, f)
    assert L.rara_peak_copy(None, None, 16, 1, None) == 1
    assert L.rara_peak_copy(ctypes.c_void_p(16), ctypes.c_void_p(16), 15, 1, None) == 1
    assert L.rara_peak_fma(None, 1, 1, None) == 1
    assert L.rara_peak_fma_flops(2, 3) == 2.0 * 16 * 256 * 2 * 3


def test_header_compiles_as_c(tmp_path):
    src = tmp_path / "t.c"
    src.write_text('#include "rara.h"\nint main(void){ rara_camera c; rara_plane p; (void)c; (void)p; '
                   'return (int)sizeof(rara_projected) == 0; }\n')
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER), str(src), "-o",
                    str(tmp_path / "t")], check=True)


def test_struct_layouts_match_header(B, tmp_path):
    """Every ctypes struct of the binding has the C header's size and field
    offsets (the binding marshals by layout)."""
    pairs = [("rara_gaussians", B.Gaussians), ("rara_camera", B.Camera), ("rara_plane", B.Plane),
             ("rara_projected", B.Projected), ("rara_binned", B.Binned), ("rara_grads", B.Grads),
             ("rara_render_item", B.RenderItem)]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "rara.h"', 'int main(void){']
    for cname, py in pairs:
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append('return 0; }')
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True)
    got = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                               check=True).stdout.splitlines())
    for cname, py in pairs:
        assert int(got[f"{cname} sizeof"]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname} {f}"]) == getattr(py, f).offset, (cname, f)


def test_status_strings_and_version(B):
    assert B.status_string(B.RARA_OK) == "ok"
    assert "invalid" in B.status_string(B.RARA_ERR_INVALID)
    assert B.status_string(99) == "unknown status"
    assert "gfx950" in B.version()


def test_workspace_sizes(B):
    assert B.workspace_bytes(B.RARA_WS_BIN_SORT, 1000, 0, 128, 128) == 0
    assert B.workspace_bytes(B.RARA_WS_BIN_SORT, -1, 10, 128, 128) == 0
    assert B.workspace_bytes(B.RARA_WS_BIN_SORT, 1000, 1 << 31, 128, 128) == 0
    a = B.workspace_bytes(B.RARA_WS_BIN_SORT, 1000, 10_000, 128, 128)
    b = B.workspace_bytes(B.RARA_WS_BIN_SORT, 1000, 100_000, 128, 128)
    assert 0 < a < b
    assert b >= 100_000 * 8      # tile keys and values of the pair sort
    assert B.workspace_bytes(7, 1000, 10_000, 128, 128) == 0


def _cam(B, w=128, h=128):
    from paper_2506_20202_amd import scenes
    return B.make_camera(scenes.tiny_camera(w, h))


def test_argument_validation_before_any_launch(B):
    lib = B.lib()
    g = B.Gaussians()
    g.n, g.sh_degree = 10, 0
    cam = _cam(B)
    pl = B.Plane()
    pl.n = (ctypes.c_float * 3)(0.0, 0.0, 1.0)
    pl.enabled = 1
    out = B.Projected()
    # null Gaussian arrays
    assert lib.rara_preprocess(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(pl), ctypes.byref(out), None) \
        == B.RARA_ERR_INVALID
    # SH degree out of range
    g.sh_degree = 4
    assert lib.rara_preprocess(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(pl), ctypes.byref(out), None) \
        == B.RARA_ERR_UNSUPPORTED
    g.sh_degree = 0
    # an SH layout other than the two the header names
    hdr = open(os.path.join(ROOT, "include", "rara.h")).read()
    assert int(re.search(r"RARA_SH_COEFF_MAJOR = (\d+)", hdr).group(1)) == B.SH_COEFF_MAJOR
    assert int(re.search(r"RARA_SH_GAUSSIAN_MAJOR = (\d+)", hdr).group(1)) == B.SH_GAUSSIAN_MAJOR
    g0 = B.Gaussians()
    for layout, want in [(B.SH_COEFF_MAJOR, B.RARA_OK), (B.SH_GAUSSIAN_MAJOR, B.RARA_OK), (2, B.RARA_ERR_INVALID),
                         (-1, B.RARA_ERR_INVALID)]:
        g0.sh_layout = layout   # n = 0: validated, then nothing to launch
        assert lib.rara_preprocess(ctypes.byref(g0), ctypes.byref(cam), ctypes.byref(pl), ctypes.byref(out),
                                   None) == want, layout
    # zero plane normal with clipping enabled
    pl0 = B.Plane()
    pl0.enabled = 1
    assert lib.rara_preprocess(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(pl0), ctypes.byref(out), None) \
        == B.RARA_ERR_INVALID
    # bad camera
    bad = _cam(B)
    bad.width = 0
    assert lib.rara_preprocess(ctypes.byref(g), ctypes.byref(bad), ctypes.byref(pl), ctypes.byref(out), None) \
        == B.RARA_ERR_INVALID
    bad = _cam(B)
    bad.near_z = 0.0
    assert lib.rara_preprocess(ctypes.byref(g), ctypes.byref(bad), ctypes.byref(pl), ctypes.byref(out), None) \
        == B.RARA_ERR_INVALID
    # negative n
    g.n = -1
    assert lib.rara_preprocess(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(pl), ctypes.byref(out), None) \
        == B.RARA_ERR_INVALID
    # n == 0 is a valid no-op
    g.n = 0
    assert lib.rara_preprocess(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(pl), ctypes.byref(out), None) \
        == B.RARA_OK
    # bin_sort: capacity and workspace checks
    bins = B.Binned()
    assert lib.rara_bin_sort(ctypes.byref(out), 10, ctypes.byref(cam), 100, None, 0, ctypes.byref(bins), None) \
        == B.RARA_ERR_INVALID
    fake = ctypes.c_void_p(0x1000)
    bins.keys = bins.vals = bins.ranges = bins.num_pairs = bins.overflow = bins.work = 0x1000
    assert lib.rara_bin_sort(ctypes.byref(out), 0, ctypes.byref(cam), 100, fake, 16, ctypes.byref(bins), None) \
        == B.RARA_ERR_INVALID   # workspace too small
    assert lib.rara_bin_sort(ctypes.byref(out), 0, ctypes.byref(cam), 0, fake, 1 << 30, ctypes.byref(bins), None) \
        == B.RARA_ERR_INVALID   # capacity < 1
    # backward: pair capacity and pair_start are required
    grads = B.Grads()
    grads.mean = grads.scale = grads.quat = grads.opacity = grads.sh = grads.plane = 0x1000
    bins.pair_start = 0
    for cap, ps in [(0, 0x1000), (1 << 30, 0x1000), (100, 0)]:
        bins.pair_start = ps
        assert lib.rara_render_backward(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(pl), (ctypes.c_float * 3)(),
                                        ctypes.byref(out), ctypes.byref(bins), cap, fake, fake, fake,
                                        ctypes.byref(grads), fake, 1 << 40, None) == B.RARA_ERR_INVALID
    bins.pair_start = 0x1000
    assert B.workspace_bytes(B.RARA_WS_BACKWARD, 1000, 0, 128, 128) == 0
    assert B.workspace_bytes(B.RARA_WS_BACKWARD, 1000, 2000, 128, 128) >= 2000 * 21 * 4
    # render: null outputs
    bg = (ctypes.c_float * 3)(0, 0, 0)
    assert lib.rara_render(ctypes.byref(out), 0, ctypes.byref(bins), ctypes.byref(cam), ctypes.byref(pl), bg, None,
                           None, None, None, None, None) == B.RARA_ERR_INVALID


def test_static_bin_sort_rejects_frames_beyond_its_workspace(B):
    """rara_bin_sort_static (the entry point for callers that cannot allocate)
    checks its arguments like rara_bin_sort and refuses a frame whose
    workspace exceeds RARA_STATIC_WS_BYTES with RARA_ERR_SCRATCH, both before
    anything reaches the GPU; the headline frame (1M Gaussians, 5M pairs of
    capacity at 1080p) fits."""
    lib = B.lib()
    hdr = open(HEADER).read()
    assert re.search(r"#define RARA_STATIC_WS_BYTES \(\(size_t\)64 << 20\)", hdr)
    assert B.STATIC_WS_BYTES == 64 << 20
    assert "RARA_ERR_SCRATCH = 5" in hdr and B.RARA_ERR_SCRATCH == 5
    assert "static workspace" in B.status_string(B.RARA_ERR_SCRATCH)
    cam = _cam(B)
    proj = B.Projected()
    proj.label = proj.splat = proj.ray = proj.depth = proj.tiles_touched = proj.tile_rec = 0x1000
    bins = B.Binned()
    assert lib.rara_bin_sort_static(ctypes.byref(proj), 10, ctypes.byref(cam), 100, ctypes.byref(bins), None) \
        == B.RARA_ERR_INVALID   # null outputs
    bins.keys = bins.vals = bins.ranges = bins.num_pairs = bins.overflow = bins.work = 0x1000
    assert lib.rara_bin_sort_static(ctypes.byref(proj), 10, ctypes.byref(cam), 0, ctypes.byref(bins), None) \
        == B.RARA_ERR_INVALID   # capacity < 1
    n, cap = 1_000_000, 10_000_000
    assert B.workspace_bytes(B.RARA_WS_BIN_SORT, n, cap, 1920, 1080) > B.STATIC_WS_BYTES
    assert lib.rara_bin_sort_static(ctypes.byref(proj), n, ctypes.byref(cam), cap, ctypes.byref(bins), None) \
        == B.RARA_ERR_SCRATCH
    assert B.workspace_bytes(B.RARA_WS_BIN_SORT, 1_000_000, 5_000_000, 1920, 1080) <= B.STATIC_WS_BYTES


def test_render_batch_validation(B):
    """rara_render_batch checks its items on the host: a count outside
    [1, RARA_MAX_BATCH], an item rara_render would reject, and a clip region
    (not supported in a batch) are refused before any launch."""
    lib = B.lib()
    assert "#define RARA_MAX_BATCH 16" in open(HEADER).read() and B.MAX_BATCH == 16
    assert lib.rara_render_batch(None, 1, None) == B.RARA_ERR_INVALID
    items = (B.RenderItem * 17)()
    assert lib.rara_render_batch(items, 0, None) == B.RARA_ERR_INVALID
    assert lib.rara_render_batch(items, 17, None) == B.RARA_ERR_INVALID
    assert lib.rara_render_batch(items, 1, None) == B.RARA_ERR_INVALID   # null pointers
    proj, bins = B.Projected(), B.Binned()
    proj.label = proj.splat = proj.ray = proj.depth = proj.tiles_touched = proj.tile_rec = 0x1000
    bins.keys = bins.vals = bins.ranges = bins.num_pairs = bins.overflow = bins.work = 0x1000
    cam = _cam(B)
    box = B.make_plane(__import__("paper_2506_20202_amd.scenes", fromlist=["x"]).box_region((-1, -1, -1), (1, 1, 1)))
    bg = (ctypes.c_float * 3)()
    it = items[0]
    it.proj, it.n, it.bins = ctypes.pointer(proj), 10, ctypes.pointer(bins)
    it.cam, it.plane, it.bg = ctypes.pointer(cam), ctypes.pointer(box), bg
    it.image = it.final_T = it.n_contrib = 0x1000
    assert lib.rara_render_batch(items, 1, None) == B.RARA_ERR_UNSUPPORTED
    bad = _cam(B)
    bad.width = 0
    it.cam = ctypes.pointer(bad)
    assert lib.rara_render_batch(items, 1, None) == B.RARA_ERR_INVALID


def test_clip_modes_agree_and_invalid_modes_are_rejected(B):
    """rara_plane.enabled values: the header, the binding and the oracle agree;
    rule 3 and flags without the RaRa rule are RARA_ERR_INVALID (checked on the
    host before any launch)."""
    hdr = open(os.path.join(ROOT, "include", "rara.h")).read()
    import oracle
    for name, ov in [("RARA_CLIP_OFF", oracle.CLIP_OFF), ("RARA_CLIP_RARA", oracle.CLIP_RARA),
                     ("RARA_CLIP_HARD", oracle.CLIP_HARD), ("RARA_CLIP_TIGHT", oracle.CLIP_TIGHT),
                     ("RARA_CLIP_STRICT_MISS", oracle.CLIP_STRICT_MISS)]:
        hv = int(re.search(name + r" = (\d+)", hdr).group(1))
        assert hv == getattr(B, name) == ov
    lib = B.lib()
    g = B.Gaussians()
    g.n = 0
    cam = _cam(B)
    out = B.Projected()
    for mode, ok in [(0, True), (1, True), (2, True), (5, True), (9, True), (13, True),
                     (3, False), (6, False), (4, False), (8, False), (16, False), (-1, False)]:
        pl = B.Plane()
        pl.n[2] = 1.0
        pl.enabled = mode
        st = lib.rara_preprocess(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(pl), ctypes.byref(out), None)
        assert st == (B.RARA_OK if ok else B.RARA_ERR_INVALID), (mode, st)


def test_clip_regions_are_validated_on_the_host(B):
    """rara_plane.count: a region of 2..RARA_MAX_PLANES half-spaces; a count
    above the maximum, a zero normal among the extra planes, or a region
    without rara_projected.ray_ext is RARA_ERR_INVALID; the backward and frame
    graphs take one plane (RARA_ERR_UNSUPPORTED).  All checked before any
    launch."""
    import oracle
    from paper_2506_20202_amd import scenes
    hdr = open(os.path.join(ROOT, "include", "rara.h")).read()
    assert int(re.search(r"#define RARA_MAX_PLANES (\d+)", hdr).group(1)) == B.MAX_PLANES == scenes.MAX_PLANES
    orc = open(os.path.join(ROOT, "oracle", "rara_oracle.c")).read()
    assert int(re.search(r"#define OR_MAX_PLANES (\d+)", orc).group(1)) == B.MAX_PLANES
    lib = B.lib()
    g = B.Gaussians()
    g.n, g.sh_degree = 0, 0
    cam = _cam(B)
    out = B.Projected()
    box = B.make_plane(scenes.box_region((-1, -1, -1), (1, 1, 1)))
    assert box.count == 6
    # n = 0 returns before launching: a valid region is accepted
    assert lib.rara_preprocess(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(box), ctypes.byref(out), None) \
        == B.RARA_OK
    for bad in (B.MAX_PLANES + 1, -1):
        pl = B.make_plane(scenes.box_region((-1, -1, -1), (1, 1, 1)))
        pl.count = bad
        assert lib.rara_preprocess(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(pl), ctypes.byref(out),
                                   None) == B.RARA_ERR_INVALID
    zero = B.make_plane(scenes.box_region((-1, -1, -1), (1, 1, 1)))
    zero.extra[2] = (ctypes.c_float * 4)(0.0, 0.0, 0.0, 1.0)
    assert lib.rara_preprocess(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(zero), ctypes.byref(out), None) \
        == B.RARA_ERR_INVALID
    # a region needs ray_ext once there are Gaussians
    g.n = 10
    fake = ctypes.c_void_p(0x1000)
    full = B.Projected()
    full.label = full.splat = full.ray = full.depth = full.tiles_touched = full.tile_rec = 0x1000
    g.mean = g.scale = g.quat = g.opacity = g.sh = 0x1000
    assert lib.rara_preprocess(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(box), ctypes.byref(full), None) \
        == B.RARA_ERR_INVALID
    # the tile records are required and 16-byte aligned (refused before any launch)
    one = B.make_plane(scenes.tiny_plane(1))
    for bad in (0, 0x1008):
        full.tile_rec = bad
        assert lib.rara_preprocess(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(one), ctypes.byref(full),
                                   None) == B.RARA_ERR_INVALID
    full.tile_rec = 0x1000
    bins = B.Binned()
    bins.keys = bins.vals = bins.ranges = bins.num_pairs = bins.overflow = bins.work = bins.pair_start = 0x1000
    img = (ctypes.c_float * 3)()
    assert lib.rara_render(ctypes.byref(full), 10, ctypes.byref(bins), ctypes.byref(cam), ctypes.byref(box), img,
                           fake, fake, fake, None, None, None) == B.RARA_ERR_INVALID
    grads = B.Grads()
    grads.mean = grads.scale = grads.quat = grads.opacity = grads.sh = grads.plane = 0x1000
    full.ray_ext = 0x1000
    assert lib.rara_render_backward(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(box), img, ctypes.byref(full),
                                    ctypes.byref(bins), 100, fake, fake, fake, ctypes.byref(grads), fake, 1 << 40,
                                    None) == B.RARA_ERR_UNSUPPORTED
    # the oracle reads the same region
    np.testing.assert_array_equal(oracle.planes_of(scenes.box_region((-1, -1, -1), (1, 1, 1)))[1:],
                                  np.array([list(r) for r in box.extra[:5]], np.float32))


def test_constants_agree_between_oracle_and_kernels():
    """The oracle and the kernels are written separately; their conventions
    (thresholds, dilation, guard band, tile size, kappa) must agree."""
    internal = open(os.path.join(ROOT, "paper_2506_20202_amd", "csrc", "rara_internal.h")).read()
    orc = open(os.path.join(ROOT, "oracle", "rara_oracle.c")).read()

    def k(name):
        return float(re.search(r"constexpr \w+ " + name + r" = ([0-9.e+-]+)", internal).group(1).rstrip("f"))

    def o(name):
        m = re.search(r"#define " + name + r" \(?([0-9.e+-]+)(?: / ([0-9.]+))?", orc)
        v = float(m.group(1))
        return v / float(m.group(2)) if m.group(2) else v

    assert k("kTile") == o("OR_TILE")
    assert abs(k("kAlphaMax") - o("OR_ALPHA_MAX")) < 1e-7
    assert k("kTMin") == o("OR_T_MIN")
    assert k("kDilation") == o("OR_DILATION")
    assert k("kGuard") == o("OR_GUARD")
    assert k("kKappa2") == 9.0
    import oracle
    assert oracle.KAPPA ** 2 == 9.0


def test_schedule_constants_agree_with_the_gpu_tests():
    """The GPU tests check the blend schedule with their own copies of the
    long-list thresholds; they must be the kernels' values."""
    internal = open(os.path.join(ROOT, "paper_2506_20202_amd", "csrc", "rara_internal.h")).read()
    from tests import gpu_helpers as H
    assert int(re.search(r"constexpr uint32_t kHeavyList = (\d+);", internal).group(1)) == H.HEAVY_LIST
    assert int(re.search(r"constexpr uint32_t kMaxUnitTiles = (\d+);", internal).group(1)) == H.MAX_UNIT_TILES
    assert int(re.search(r"constexpr uint32_t kUnitBucket = (\d+);", internal).group(1)) == H.UNIT_BUCKET


def test_unit_threshold_takes_the_longest_lists():
    """The schedule's unit class is the up to 512 longest long lists, to a
    bucket of 128 entries: all long lists when there are at most 512; else a
    threshold that at most 512 reach and the next bucket down would exceed."""
    import numpy as np
    from tests import gpu_helpers as H
    assert H.unit_threshold(np.array([5, 1500, 3000])) == H.HEAVY_LIST
    rng = np.random.default_rng(0)
    counts = rng.integers(0, 9000, 8160)
    L = H.unit_threshold(counts)
    assert (counts >= L).sum() <= 512 < (counts >= L - H.UNIT_BUCKET).sum()
    assert H.unit_threshold(np.full(600, 40000)) == np.inf   # the last bucket alone holds more than 512


def test_sh_constants_agree_with_closed_forms():
    """The kernel's SH normalisations (decimal literals) equal the closed forms
    the oracle evaluates."""
    src = open(os.path.join(ROOT, "paper_2506_20202_amd", "csrc", "preprocess.hip")).read()
    lits = sorted(set(float(x) for x in re.findall(r"(\d\.\d{10,})", src)))
    forms = sorted(set([np.sqrt(1 / (4 * np.pi)), np.sqrt(3 / (4 * np.pi)), np.sqrt(15 / (4 * np.pi)),
                        np.sqrt(5 / (16 * np.pi)), np.sqrt(15 / (16 * np.pi)), np.sqrt(35 / (32 * np.pi)),
                        np.sqrt(105 / (4 * np.pi)), np.sqrt(21 / (32 * np.pi)), np.sqrt(7 / (16 * np.pi)),
                        np.sqrt(105 / (16 * np.pi))]))
    assert len(lits) == len(forms)
    np.testing.assert_allclose(lits, forms, rtol=1e-15)


def test_product_path_fails_loudly_without_library(monkeypatch):
    from paper_2506_20202_amd import binding
    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(binding, "LIB_PATH", "/nonexistent/librara.so")
    with pytest.raises(RuntimeError, match="not built"):
        binding.lib()
