"""Throughput benchmark of the hybrid multi-resolution frame on one MI355X.

One step = one 720p hybrid frame of the textured procedural ~100k-triangle
scene: HRLS 1280x720 at 4 spp with albedo/normal/depth, LRHS 320x180 at 64 spp
(max depth 8, Russian roulette from vertex 3; 7,372,800 paths, spp_avg =
64/16 + 4 = 8) and the BF16 fusion network on both.  Inputs (scene, LBVH,
weights) are resident in HBM before timing starts.  The timed frames run as a
stream of frames on one stream, each frame's fusion overlapping the next
frame's render (every frame's whole work is inside the timed region); the
same frames one at a time are reported beside it.

Prints one JSON line: Mpaths/s of the frame, ms per frame, the roofline
position of the dominant kernel (timed live with HIP events on its launch
stream), the equal-PSNR comparison with plain renders (PSNR against an
independent 1024-spp reference), and the FP64 oracle timed on the host cores.
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

METRIC = "Mpaths/s; ms/720p frame hybrid (4spp+LRHS+CNN) vs plain spp at equal PSNR"
HRLS = (1280, 720, 4)
LRHS = (320, 180, 64)
MAX_DEPTH = 8
SCENE_SEED = 7
PEAK_FP32_TFLOPS = 157.3  # MI355X vector FP32 (FMA = 2 FLOP, packed)
# Algorithmic FP32 operations (FMA counted as 2) of the closest-hit traversal:
#   per BVH4 node visit: four slab tests (6 FMA, 10 min/max, 1 scale, 2 compares each = 25)
#     + a 5-comparator sorting network on the entry distances = 105
#   per triangle test: Moller-Trumbore (2 cross, 4 dot, 3 sub, 1 rcp, 3 scale, 7 compares) = 52
#   per ray: reciprocal direction and scaled origin = 10
FLOP_PER_VISIT = 105
FLOP_PER_TEST = 52
FLOP_PER_RAY = 10
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "extend_procedural101k_720p_traffic.txt")
WEIGHTS = os.path.join(ROOT, "paper_2106_12802_amd", "weights", "fusion_l1_textured.bin")
# the paper's own network (x4), trained on the same synthetic pairs
WEIGHTS_RDG = os.path.join(ROOT, "paper_2106_12802_amd", "weights", "fusion_rdg_l1.bin")
# the 16-block trunk trained with a random spp pair per iteration
WEIGHTS_RSPP = os.path.join(ROOT, "paper_2106_12802_amd", "weights", "fusion_l1_random_spp.bin")
PEAK_BF16_TFLOPS = 2500.0  # MI355X dense BF16 MFMA
CNN_FLOP_720P = 175.7e9    # 87.85 GMAC per 720p frame
# the paper's network on a 1024x1024 image, seconds (its runtime table; Titan Xp)
PAPER_TABLE5_S = {2: 0.362, 4: 0.118, 8: 0.052}


def rdg_flop(H, W, scale=4):
    """Forward FLOP of the paper's network (residual dense groups) at x`scale` on
    one H x W frame: 2 x sum over convs of pixels x C_out x C_in x k^2."""
    D = {2: 1, 4: 2, 8: 3}[scale]
    p = H * W // scale ** 2  # LR pixels
    mac = (scale ** 2 * p * 64 * 10 * 9 + p * 64 * 3 * 9 + p * 64 * (64 + 64 * 4 ** D)
           + 15 * p * 64 * 9 * (64 + 128 + 192 + 256)                  # 15 dense blocks
           + sum(4 ** k * p * 256 * 64 * 9 for k in range(D))          # upscaling steps
           + scale ** 2 * p * 3 * 64 * 9)                              # reconstruction
    return 2 * mac


# the traversal kernel and the BVH builder (the tree decides what a launch reads)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2106_12802_amd", "csrc", f)
                  for f in ("trace.hip", "lbvh.hip")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic():
    """HBM bytes per extend launch from the committed rocprofv3 PMC summary, if current."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    vals = {}
    for line in open(TRAFFIC_SUMMARY):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_sources_sha256_16") != kernel_source_hash():
        return None  # the kernel changed since the counters were taken
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


COPY_BYTES = 1 << 30  # plain device copy used to calibrate the PMC byte counters


def copy_calibration():
    """One plain 1 GiB device-to-device copy (reads and writes COPY_BYTES)."""
    import torch
    src = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def _pmc_rows(path):
    import csv
    files = [path] if os.path.isfile(path) else [
        os.path.join(dp, f) for dp, _, fs in os.walk(path) for f in fs
        if f.endswith("counter_collection.csv")]
    rows = []
    for fn in files:
        with open(fn) as f:
            rows += list(csv.DictReader(f))
    return rows


def pmc_summary(fetch_path, write_path, out_path):
    """Turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch) into the
    HBM traffic summary read by read_traffic()."""
    def per_kernel(path, counter):
        acc = {}
        for r in _pmc_rows(path):
            if r.get("Counter_Name") != counter:
                continue
            acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return acc

    fetch = per_kernel(fetch_path, "FETCH_SIZE")
    write = per_kernel(write_path, "WRITE_SIZE")

    def copy_value(d):
        cands = [(max(v), k) for k, v in d.items() if "copy" in k.lower()]
        return max(cands)[0] if cands else None

    cf, cw = copy_value(fetch), copy_value(write)
    fs = COPY_BYTES / (cf * 1024.0) if cf else None
    ws = COPY_BYTES / (cw * 1024.0) if cw else None
    ext = [k for k in fetch if is_extend(k)]
    if not ext or fs is None or ws is None:
        raise SystemExit(f"pmc summary: missing kernels (extend {ext}, copy {cf}, {cw})")
    fv = [x for k in ext for x in fetch[k]]
    wv = [x for k in ext for x in write.get(k, [])]
    f_kib = sum(fv) / len(fv)
    w_kib = sum(wv) / max(len(wv), 1)
    hbm = f_kib * 1024.0 * fs + w_kib * 1024.0 * ws
    lines = [
        "# HBM traffic per closest-hit launch (k_extend_wave at bounce 0 and k_extend<false,",
        "# false> at bounces 1-2, averaged over their dispatches), procedural scene seed 7",
        "# (101,446 triangles, textured), 720p hybrid frame HRLS 1280x720@4 + LRHS 320x180@64",
        "# (max depth 8) + fusion network.",
        "# Made by (each pass its own process, run from the repository root):",
        "#   rocprofv3 --pmc FETCH_SIZE -f csv -d gpurun_out/pmc_fetch -o pmc -- python bench.py "
        "--steps 1 --warmup 0 --no-cpu-baseline --equal-psnr-scenes 0 --batch-scenes 0 --no-paper-net --no-mis --no-camera --no-spp-pairs --no-two-calls --no-training --no-ablations "
        "--copy-calibration",
        "#   rocprofv3 --pmc WRITE_SIZE -f csv -d gpurun_out/pmc_write -o pmc -- python bench.py "
        "--steps 1 --warmup 0 --no-cpu-baseline --equal-psnr-scenes 0 --batch-scenes 0 --no-paper-net --no-mis --no-camera --no-spp-pairs --no-two-calls --no-training --no-ablations "
        "--copy-calibration",
        "#   python bench.py --pmc-summary gpurun_out/pmc_fetch gpurun_out/pmc_write",
        "# Counters are KiB per dispatch; each is scaled by COPY_BYTES over what the same counter",
        "# reads for a plain 1 GiB device copy in the same process.",
        f"copy_bytes = {COPY_BYTES}",
        f"copy_fetch_kib = {cf:.1f}",
        f"copy_write_kib = {cw:.1f}",
        f"fetch_scale = {fs:.4f}",
        f"write_scale = {ws:.4f}",
        f"extend_dispatches = {len(fv)}",
        f"extend_fetch_kib_per_dispatch = {f_kib:.1f}",
        f"extend_write_kib_per_dispatch = {w_kib:.1f}",
        f"hbm_bytes_per_launch = {hbm:.0f}",
        f"kernel_sources_sha256_16 = {kernel_source_hash()}",
    ]
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


COUNTERS_SUMMARY = os.path.join(ROOT, "profiles", "hybrid_frame_procedural101k_720p_counters.txt")
# the kernels the counters describe and the sources that make them
COUNTER_SOURCES = [os.path.join(ROOT, "paper_2106_12802_amd", "csrc", f)
                   for f in ("trace.hip", "lbvh.hip", "cnn.hip", "net.hip")]
PROFILE_ARGS = ("--steps 1 --warmup 0 --no-cpu-baseline --equal-psnr-scenes 0 --batch-scenes 0 "
                "--no-paper-net --no-mis --no-camera --no-spp-pairs --no-two-calls --no-training --no-ablations")
# rocprofv3 --pmc passes (one process each; each within the per-block counter limits)
COUNTER_PASSES = {
    "valu": "VALUBusy VALUUtilization SQ_INSTS_VALU SQ_WAVES GRBM_GUI_ACTIVE",
    "cache": "TCC_HIT_sum TCC_MISS_sum TCP_TOTAL_CACHE_ACCESSES_sum TCP_TCC_READ_REQ_sum "
             "GRBM_GUI_ACTIVE",
    "mfma": "MfmaUtil SQ_INSTS_VALU_MFMA_MOPS_BF16 SQ_LDS_BANK_CONFLICT SQ_LDS_IDX_ACTIVE "
            "SQ_BUSY_CYCLES GRBM_GUI_ACTIVE",
}
# kernel (a prefix of its demangled name, after the namespace) -> short name
# (rocprofv3 name prefix once "void ", "mrs::" and the anonymous namespace are
# dropped; short name)
COUNTER_KERNELS = [("k_extend_wave", "k_extend_wave"), ("k_extend<false,", "k_extend"),
                   ("k_shadow<false,", "k_shadow"), ("k_tail<false,", "k_tail"),
                   ("k_shade", "k_shade"), ("k_res_block", "k_res_block"),
                   ("k_conv3_lds<64, 4, 16, false>", "k_conv3_lds<64,4,16>"),
                   ("k_conv3_lds<16, 4, 16, false>", "k_conv3_lds<16,4,16>"),
                   ("k_conv3_lds<8, 4, 16, false>", "k_conv3_lds<8,4,16>"),
                   ("k_conv3_lds<80, 1, 16, false>", "k_conv3_lds<80,1,16>"),
                   ("k_conv<4>", "k_conv<4>")]
# the closest-hit launches bench.py times as "extend": bounce 0 a wave at a time,
# the other wavefront bounces lane by lane (k_extend<true, ..> is the counting pass)
EXTEND_KERNELS = ("k_extend_wave", "k_extend<false,")


def is_extend(name):
    n = name.replace("void ", "").replace("(anonymous namespace)::", "").replace("mrs::", "")
    return any(n.startswith(pre) for pre in EXTEND_KERNELS)


def counter_source_hash() -> str:
    h = hashlib.sha256()
    for path in COUNTER_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counters_summary(dirs, out_path):
    """Per-kernel figures from the rocprofv3 --pmc passes of COUNTER_PASSES (their
    output directories, in that order): each counter summed over a kernel's
    dispatches, percentages weighted by each dispatch's GRBM_GUI_ACTIVE cycles."""
    import re
    vals = {}   # short kernel name -> counter -> [sum over dispatches]
    gui = {}    # (pass, kernel) -> total active cycles
    disp = {}
    for (pname, _), d in zip(COUNTER_PASSES.items(), dirs):
        per = {}
        for r in _pmc_rows(d):
            name = r["Kernel_Name"].replace("void ", "").replace(
                "(anonymous namespace)::", "").replace("mrs::", "")
            short = next((sh for pre, sh in COUNTER_KERNELS if name.startswith(pre)), None)
            if short is None:
                continue
            key = (short, r.get("Dispatch_Id") or r.get("Correlation_Id"))
            cs = per.setdefault(key, {})
            cs[r["Counter_Name"]] = float(r["Counter_Value"])
            cs["_ns"] = float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
        for (short, _), cs in per.items():
            g = cs.pop("_ns")  # the dispatch's duration (ns) weighs its percentages
            gui[(pname, short)] = gui.get((pname, short), 0.0) + g
            disp[(pname, short)] = disp.get((pname, short), 0) + 1
            v = vals.setdefault(short, {})
            for c, x in cs.items():
                if c in ("VALUBusy", "VALUUtilization", "MfmaUtil"):
                    v[c] = v.get(c, 0.0) + x * g  # weighted, divided below
                else:
                    v[c] = v.get(c, 0.0) + x
    lines = [
        "# Hardware counters of the 720p hybrid frame's kernels (procedural scene seed 7,",
        "# 101,446 triangles; HRLS 1280x720@4 + LRHS 320x180@64, depth 8; BF16 fusion network):",
        "# one counting frame (k_*<true>, not listed), one pipelined frame and the network once",
        "# alone.  Made by (one process per pass, from the repository root, cd /tmp first):",
    ]
    for pname, ctrs in COUNTER_PASSES.items():
        lines.append(f"#   rocprofv3 --pmc {ctrs} -f csv -d gpurun_out/pmc_{pname} -o pmc -- "
                     f"python bench.py {PROFILE_ARGS}")
    lines += ["#   python bench.py --counters-summary gpurun_out/pmc_valu gpurun_out/pmc_cache "
              "gpurun_out/pmc_mfma",
              "# Sums over each kernel's dispatches; VALUBusy / VALUUtilization / MfmaUtil are",
              "# rocprofv3's derived percentages, weighted by each dispatch's duration (its",
              "# start and end timestamps; counter runs serialise the dispatches).",
              "# L1 hit = 1 - TCP_TCC_READ_REQ / TCP_TOTAL_CACHE_ACCESSES; L2 hit = TCC_HIT /",
              "# (TCC_HIT + TCC_MISS); VALU insts per wave = SQ_INSTS_VALU / SQ_WAVES;",
              "# BF16 TFLOP/s = 512 SQ_INSTS_VALU_MFMA_MOPS_BF16 / the dispatches' duration.",
              f"kernel_sources_sha256_16 = {counter_source_hash()}", ""]
    for _, short in COUNTER_KERNELS:
        v = vals.get(short)
        if not v:
            continue
        out = []
        gv, gc, gm = (gui.get((p, short), 0.0) for p in COUNTER_PASSES)
        if gv > 0 and "VALUBusy" in v:
            out.append(f"valu_busy_pct = {v['VALUBusy'] / gv:.2f}")
            out.append(f"valu_lane_util_pct = {v['VALUUtilization'] / gv:.2f}")
            out.append(f"valu_insts_per_wave = {v['SQ_INSTS_VALU'] / max(v['SQ_WAVES'], 1):.1f}")
        if "TCP_TOTAL_CACHE_ACCESSES_sum" in v:
            acc, miss = v["TCP_TOTAL_CACHE_ACCESSES_sum"], v["TCP_TCC_READ_REQ_sum"]
            out.append(f"l1_hit = {1.0 - miss / max(acc, 1):.4f}")
            h, m = v["TCC_HIT_sum"], v["TCC_MISS_sum"]
            out.append(f"l2_hit = {h / max(h + m, 1):.4f}")
        if gm > 0 and "MfmaUtil" in v:
            out.append(f"mfma_util_pct = {v['MfmaUtil'] / gm:.2f}")
            tf = 512.0 * v["SQ_INSTS_VALU_MFMA_MOPS_BF16"] / (gm * 1e-9) / 1e12
            out.append(f"mfma_bf16_tflops = {tf:.1f}")
            li = v.get("SQ_LDS_IDX_ACTIVE", 0.0)
            if li > 0:
                out.append(f"lds_bank_conflict_per_access_cycle = "
                           f"{v['SQ_LDS_BANK_CONFLICT'] / li:.4f}")
        out.append(f"dispatches = {max(disp.get((p, short), 0) for p in COUNTER_PASSES)}")
        out.append(f"us_per_dispatch = {gv / max(disp.get(('valu', short), 1), 1) / 1e3:.1f}")
        lines += [f"[{short}]"] + out + [""]
    with open(out_path, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


def read_counters():
    """{kernel: {figure: value}} from the committed counter summary, if it belongs to
    the current kernel sources (None otherwise)."""
    if not os.path.exists(COUNTERS_SUMMARY):
        return None
    res, cur, sha = {}, None, None
    for line in open(COUNTERS_SUMMARY):
        line = line.strip()
        if line.startswith("kernel_sources_sha256_16"):
            sha = line.split("=", 1)[1].strip()
        elif line.startswith("[") and line.endswith("]"):
            cur = res.setdefault(line[1:-1], {})
        elif "=" in line and cur is not None and not line.startswith("#"):
            k, v = line.split("=", 1)
            cur[k.strip()] = float(v)
    return res if sha == counter_source_hash() else None


STATS_SUMMARY = os.path.join(ROOT, "profiles", "hybrid_frame_procedural101k_720p_kernel_stats.txt")
STATS_CMD = ("rocprofv3 --kernel-trace --stats -f csv -d gpurun_out/prof -o bench -- python -u "
             "bench.py --steps 5 --warmup 1 --no-cpu-baseline --equal-psnr-scenes 0 --batch-scenes 0 --no-paper-net --no-mis --no-camera --no-spp-pairs --no-two-calls --no-training --no-ablations")


def stats_summary(prof_dir, out_path):
    """Short text form of a rocprofv3 --stats run (kernel, calls, total, average, share)."""
    import csv
    import glob
    import re
    paths = glob.glob(os.path.join(prof_dir, "**", "*kernel_stats.csv"), recursive=True)
    if not paths:
        raise SystemExit(f"stats summary: no kernel_stats.csv under {prof_dir}")
    rows = list(csv.DictReader(open(paths[0])))

    def short(n):
        n = n.replace("mrs::(anonymous namespace)::", "").replace("void ", "")
        m = re.match(r"([\w:]+(<[^>]*>)?)", n)
        return m.group(1) if m else n[:40]

    lines = ["# 720p hybrid frame (procedural 101,446 triangles, textured; HRLS 1280x720@4 + LRHS "
             "320x180@64 as one two-job batch, depth 8; BF16 fusion network): 1 counting frame "
             "(k_*<true>) + 1 warmup + 5 timed frames, pipelined, then the network 5 times "
             "alone (k_extend_wave and k_extend<false, false>: the launches of the warmup and "
             "timed frames, whose extend average bench.py reports)",
             f"# command (from the repository root): {STATS_CMD}",
             "#   then: python bench.py --stats-summary gpurun_out/prof",
             "# rocprofv3 kernel stats: name | calls | total ms | average us | percent", ""]
    for r in rows:
        lines.append(f"{short(r['Name']):34s} | {int(r['Calls']):5d} | "
                     f"{int(r['TotalDurationNs']) / 1e6:9.3f} | {float(r['AverageNs']) / 1e3:10.2f} | "
                     f"{float(r['Percentage']):6.2f}")
    ext = [r for r in rows if is_extend(r["Name"])]
    if ext:
        calls = sum(int(r["Calls"]) for r in ext)
        tot = sum(int(r["TotalDurationNs"]) for r in ext)
        lines += ["", "# the launches bench.py's roofline averages (k_extend_wave + k_extend<false, false>):",
                  f"{'extend (all timed launches)':34s} | {calls:5d} | {tot / 1e6:9.3f} | "
                  f"{tot / max(calls, 1) / 1e3:10.2f} |"]
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def cpu_baseline(scene, threads):
    """The FP64 oracle on the host, the whole hybrid frame: its two renders and the
    FP64 network on the full 1280x720 frame (inputs: the oracle's own renders)."""
    import numpy as np
    from oracle import cnn, tracer as orc
    osc = orc.OracleScene(scene)
    t0 = time.perf_counter()
    hr = osc.render(*HRLS[:2], HRLS[2], MAX_DEPTH, 2 * SCENE_SEED, nthreads=threads, want_aux=True)
    lr = osc.render(*LRHS[:2], LRHS[2], MAX_DEPTH, 2 * SCENE_SEED + 1, nthreads=threads,
                    want_aux=False)
    t_render = time.perf_counter() - t0
    rgb = hr["rgb"].reshape(1, HRLS[1], HRLS[0], 3)
    aux = hr["aux"].reshape(1, HRLS[1], HRLS[0], 7)
    lrgb = lr["rgb"].reshape(1, LRHS[1], LRHS[0], 3)
    params = np.random.default_rng(0).uniform(-0.05, 0.05, cnn.num_params())
    t0 = time.perf_counter()
    cnn.forward(params, rgb, aux, lrgb)
    t_cnn = time.perf_counter() - t0
    paths = HRLS[0] * HRLS[1] * HRLS[2] + LRHS[0] * LRHS[1] * LRHS[2]
    total = t_render + t_cnn
    # the small case (Cornell box 64x64 @16 spp, depth 4: 65,536 paths) on one thread and on all
    from mrs_inputs import scenes as S
    small = orc.OracleScene(S.cornell(1))
    small_rate = {}
    for n in (1, threads):
        t0 = time.perf_counter()
        small.render(64, 64, 16, 4, 1001, nthreads=n)
        small_rate[f"threads_{n}"] = round(65536 / (time.perf_counter() - t0) / 1e6, 4)
    return {"value": round(paths / total / 1e6, 4), "unit": "Mpaths/s", "cores": threads,
            "host_cpus": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)),
            "small_case_mpaths_per_s": small_rate,
            "kind": "oracle",
            "sample": f"the whole frame: FP64 renders (HRLS {HRLS[0]}x{HRLS[1]}@{HRLS[2]} + LRHS "
                      f"{LRHS[0]}x{LRHS[1]}@{LRHS[2]}, {paths} paths: {t_render:.1f} s) and the "
                      f"FP64 network on the full frame ({t_cnn:.1f} s; numpy BLAS threads)",
            "render_s": round(t_render, 2), "network_s": round(t_cnn, 2),
            "ms_per_frame": round(total * 1e3, 1)}


def equal_psnr_block(net, n_scenes, log):
    """Hybrid vs plain renders at equal PSNR on the bench scene and held-out scenes;
    the same frames with the paper's own network too when its trained weights exist."""
    from mrs_inputs import scenes as S
    from paper_2106_12802_amd import hybrid as HY
    from paper_2106_12802_amd import tracer as R
    import paper_2106_12802_amd as mrs
    extra = {}
    if os.path.exists(WEIGHTS_RDG):
        extra["paper_net"] = mrs.FusionNet(arch="rdg")
        extra["paper_net"].load_weights(WEIGHTS_RDG)
    specs = [("bench", S.procedural(SCENE_SEED))]
    specs += [(f"heldout_{s}", S.procedural_sized(s, t))
              for s, t in S.training_scene_specs(200, n_scenes)]
    rows = []
    for name, scene in specs:
        gs = R.GpuScene(scene)
        r = HY.evaluate_scene(gs, net, HRLS[0], HRLS[1], seed=len(rows),
                              plain_spp=(4, 8, 16, 32, 64, 128, 256, 512), reps=2,
                              extra_nets=extra)
        gs.close()
        row = {"scene": name, "triangles": scene.num_tris,
               "psnr_hybrid": round(r["hybrid"]["psnr"], 3), "ms_hybrid": round(r["hybrid"]["ms"], 3),
               "psnr_lrhs_bilinear": round(r["lrhs_bilinear"]["psnr"], 3),
               "psnr_hrls_4spp": round(r["hrls_4spp"]["psnr"], 3),
               "plain": [[n, round(p, 3), round(t, 3)] for n, p, t in r["plain"]]}
        eq = r["equal_psnr"]
        row["equal_psnr_spp"] = None if eq is None else round(eq["spp"], 2)
        row["plain_ms_at_equal_psnr"] = None if eq is None else round(eq["ms"], 3)
        row["ratio"] = None if eq is None else round(eq["ratio"], 4)
        p64 = [t for n, p, t in r["plain"] if n == 64][0]
        row["ratio_vs_plain64"] = round(r["hybrid"]["ms"] / p64, 4)
        for k, v in r["extra"].items():
            e = v["equal_psnr"]
            row[k] = {"psnr_hybrid": round(v["psnr"], 3), "ms_hybrid": round(v["ms"], 3),
                      "equal_psnr_spp": None if e is None else round(e["spp"], 2),
                      "ratio": None if e is None else round(e["ratio"], 4)}
            log(f"[bench] {name} with the paper's network: {row[k]}")
        rows.append(row)
        log(f"[bench] {name}: hybrid {row['psnr_hybrid']} dB in {row['ms_hybrid']} ms; "
            f"equal-PSNR plain spp {row['equal_psnr_spp']} ({row['plain_ms_at_equal_psnr']} ms), "
            f"ratio {row['ratio']}")
    ratios = [r["ratio"] for r in rows if r["ratio"] is not None]
    for other in extra.values():
        other.close()
    extra_means = {}
    for k in extra:
        rk = [r[k]["ratio"] for r in rows if r[k]["ratio"] is not None]
        extra_means[f"mean_ratio_{k}"] = round(sum(rk) / len(rk), 4) if rk else None
    return {"reference": "1024 spp, independent seed, FP64 pixel sums",
            **extra_means,
            "protocol": "PSNR_N of plain renders N in 4..512 spp interpolated linearly in log2 N; "
                        "time interpolated linearly in N; ratio = hybrid ms / plain ms at equal PSNR",
            "mean_ratio": round(sum(ratios) / len(ratios), 4) if ratios else None,
            "scenes": rows}


def batched_block(net, log, n_scenes=32, tune=True):
    """Uneven render+fuse frames (32 seeded scenes, 256x256..1920x1080, 10k..1M
    triangles, HRLS 1..8 spp, LRHS 16..128 spp) as one batch plus the fusions,
    captured in a HIP graph; timed against the same frames one call at a time."""
    import torch

    import paper_2106_12802_amd as mrs
    from paper_2106_12802_amd import autotune
    from paper_2106_12802_amd import tracer as R
    from mrs_inputs import scenes as S

    t0 = time.perf_counter()
    specs = S.batch_specs(500, n_scenes)
    scenes, frames, jobs = [], [], []
    for seed, tris, W, H, sh, sl in specs:
        gs = mrs.GpuScene(S.procedural_sized(seed, tris))
        scenes.append(gs)
        f = dict(W=W, H=H, sh=sh, sl=sl, seed=seed,
                 hr=torch.empty(H, W, 3, device="cuda"), aux=torch.empty(H, W, 7, device="cuda"),
                 lr=torch.empty(H // 4, W // 4, 3, device="cuda"),
                 out=torch.empty(H, W, 3, device="cuda"))
        frames.append(f)
        jobs.append(dict(scene=gs, W=W, H=H, spp=sh, max_depth=MAX_DEPTH, seed=2 * seed,
                         out_rgb=f["hr"], out_aux=f["aux"]))
        jobs.append(dict(scene=gs, W=W // 4, H=H // 4, spp=sl, max_depth=MAX_DEPTH,
                         seed=2 * seed + 1, out_rgb=f["lr"], want_aux=False))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    paths = sum(j["W"] * j["H"] * j["spp"] for j in jobs)
    log(f"[batch] {n_scenes} scenes, {paths / 1e6:.1f} M paths per batch (setup {setup_s:.1f} s)")

    def sequential():
        for gs, f in zip(scenes, frames):
            R.render_ex(gs, f["W"], f["H"], f["sh"], MAX_DEPTH, 2 * f["seed"], f["hr"], f["aux"])
            R.render_ex(gs, f["W"] // 4, f["H"] // 4, f["sl"], MAX_DEPTH, 2 * f["seed"] + 1,
                        f["lr"], None)
            net.fuse(f["hr"], f["aux"], f["lr"], out=f["out"])

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / reps

    seq_ms = timed(sequential, 2)
    seq_out = [f["out"].clone() for f in frames]
    log(f"[batch] one call per render/fuse: {seq_ms:.1f} ms")
    # autotune the batch's launch shape (each candidate gets its own batch)
    old = R.get_tuning()
    made = {}

    def workload():
        key = tuple(R.get_tuning().values())
        if key not in made:
            for b in made.values():
                b.close()
            made.clear()
            made[key] = mrs.Batch(jobs)
        made[key].render()

    tuned = None
    if tune:
        cands = [(c, b, 0) for c in (1 << 22, 1 << 23, 1 << 24, 1 << 25) for b in (4096, 8192)]
        cands.append((1 << 24, 4096, 1))
        tuned = autotune.tune(workload, f"batch{n_scenes}", "/tmp/mrs_autotune_bench.json",
                              reps=2, candidates=cands, force=True, log=log)
    for b in made.values():
        b.close()
    made.clear()
    batch = mrs.Batch(jobs)  # created under the chosen tuning
    R.set_tuning(**old)
    # capture batch + fusions in one graph, on a stream that ran them once
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())

    def frame_all():
        batch.render()
        for f in frames:
            net.fuse(f["hr"], f["aux"], f["lr"], out=f["out"])

    with torch.cuda.stream(st):
        frame_all()
    torch.cuda.synchronize()
    eager = [f["out"].clone() for f in frames]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        frame_all()
    graph_ms = timed(g.replay, 5)
    same = all(torch.equal(f["out"], e) for f, e in zip(frames, eager))
    same_seq = all(torch.equal(f["out"], e) for f, e in zip(frames, seq_out))
    log(f"[batch] batch + fusions as one HIP graph: {graph_ms:.1f} ms "
        f"({paths / graph_ms / 1e3:.1f} Mpaths/s), replay == eager: {same}, "
        f"== one call at a time: {same_seq}")
    batch.close()
    return {"workload": f"{n_scenes} procedural scenes (seeds 500.., 10k-1M triangles, "
                        "256x256-1920x1080), HRLS 1-8 spp + LRHS 16-128 spp at 1/4 size, "
                        "max depth 8, plus one fusion per frame",
            "triangles_total": int(sum(gs.num_tris for gs in scenes)), "paths": int(paths),
            "ms_sequential_calls": round(seq_ms, 3), "ms_batched_graph": round(graph_ms, 3),
            "mpaths_per_s_batched": round(paths / graph_ms / 1e3, 2),
            "speedup": round(seq_ms / graph_ms, 4), "replay_equals_eager": bool(same),
            "equals_one_call_at_a_time": bool(same_seq),
            "tuning": {k: tuned[k] for k in autotune.KEYS} if tuned else None}


def mis_block(gs, log, reps=5):
    """Multiple importance sampling of the quad lights (render option mis) on the
    bench scene: time of the two renders of the hybrid frame with and without it,
    and the PSNR of the 4-spp HRLS image against a 1024-spp reference (MIS, FP64
    pixel sums, independent seed) with and without it."""
    import torch
    from paper_2106_12802_amd import metrics as M
    from paper_2106_12802_amd import tracer as R
    (Wh, Hh, sh), (Wl, Hl, sl) = HRLS, LRHS
    ref, _ = R.render(gs, Wh, Hh, 1024, MAX_DEPTH, 1 << 41, want_aux=False, mis=True)
    res = {"reference": "1280x720 at 1024 spp with mis, FP64 pixel sums, seed 2^41"}
    # a glossy floor mirroring three quad lights: where the two strategies differ most
    from mrs_inputs import scenes as S
    glossy = R.GpuScene(S.glossy_lights(0.05))
    gref, _ = R.render(glossy, 512, 288, 4096, MAX_DEPTH, 1 << 41, want_aux=False, mis=True)
    for mis in (False, True):
        p = [M.image_metrics(R.render(glossy, 512, 288, 4, MAX_DEPTH, 200 + k, want_aux=False,
                                      mis=mis)[0], gref)["psnr"] for k in range(4)]
        res[f"glossy_psnr_4spp_{'mis' if mis else 'nee'}"] = round(sum(p) / len(p), 3)
    glossy.close()
    log(f"[bench] glossy floor 512x288 at 4 spp: NEE {res['glossy_psnr_4spp_nee']} dB, "
        f"MIS {res['glossy_psnr_4spp_mis']} dB")
    for mis in (False, True):
        hr = torch.empty(Hh, Wh, 3, device="cuda")
        lr = torch.empty(Hl, Wl, 3, device="cuda")

        def frame(i):
            R.render_ex(gs, Wh, Hh, sh, MAX_DEPTH, 2 * i, hr, None, mis=mis)
            R.render_ex(gs, Wl, Hl, sl, MAX_DEPTH, 2 * i + 1, lr, None, mis=mis)
        frame(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(reps):
            frame(i)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        psnr = [M.image_metrics(R.render(gs, Wh, Hh, sh, MAX_DEPTH, 100 + k, want_aux=False,
                                          mis=mis)[0], ref)["psnr"] for k in range(4)]
        key = "mis" if mis else "nee"
        res[f"ms_two_renders_{key}"] = round(ms, 4)
        res[f"psnr_hrls_4spp_{key}"] = round(sum(psnr) / len(psnr), 3)
        log(f"[bench] {key}: two renders {ms:.3f} ms, HRLS 4 spp PSNR {res[f'psnr_hrls_4spp_{key}']} dB")
    return res


def camera_block(gs, log, reps=5):
    """Depth of field (thin lens) and motion blur (camera translated over the
    shutter) on the bench scene: time of the two renders of the hybrid frame
    (HRLS 1280x720@4 + LRHS 320x180@64) with each effect, against the pinhole
    camera.  Lens: radius 0.15, focus 8.0 along the view axis; motion: the camera
    moves by (0.4, 0, 0) over the shutter."""
    import torch
    from paper_2106_12802_amd import tracer as R
    (Wh, Hh, sh), (Wl, Hl, sl) = HRLS, LRHS
    paths = Wh * Hh * sh + Wl * Hl * sl
    lens = {"lens_radius": 0.15, "focus_dist": 8.0}
    motion = {"cam_motion": (0.4, 0.0, 0.0)}
    cases = (("pinhole", {}), ("lens", lens), ("motion", motion), ("lens_motion", {**lens, **motion}))
    hr = torch.empty(Hh, Wh, 3, device="cuda")
    lr = torch.empty(Hl, Wl, 3, device="cuda")
    res = {"workload": "bench scene, HRLS 1280x720@4 + LRHS 320x180@64 as two render calls; "
                       "lens radius 0.15 focused at 8.0, camera motion (0.4, 0, 0)"}
    for name, kw in cases:
        def frame(i):
            R.render_ex(gs, Wh, Hh, sh, MAX_DEPTH, 2 * i, hr, None, **kw)
            R.render_ex(gs, Wl, Hl, sl, MAX_DEPTH, 2 * i + 1, lr, None, **kw)
        frame(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(reps):
            frame(i)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        res[f"ms_two_renders_{name}"] = round(ms, 4)
        res[f"mpaths_per_s_{name}"] = round(paths / ms / 1e3, 1)
        log(f"[bench] camera {name}: two renders {ms:.3f} ms")
    return res


def layers_block(gs, log, reps=5):
    """Render layers (Sec. 3.1, Eqs. 1-2: emission, diffuse, glossy) of the HRLS
    render (1280x720@4) on the bench scene: its time with the nine layer sums
    against the plain render."""
    import torch
    from paper_2106_12802_amd import tracer as R
    Wh, Hh, sh = HRLS
    hr = torch.empty(Hh, Wh, 3, device="cuda")
    lay = torch.empty(Hh, Wh, 9, device="cuda")
    res = {"workload": "bench scene, HRLS 1280x720@4 as one render call, with and without "
                       "the emission / diffuse / glossy layers"}
    for name, kw in (("plain", {}), ("layers", {"out_layers": lay})):
        R.render_ex(gs, Wh, Hh, sh, MAX_DEPTH, 0, hr, None, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(reps):
            R.render_ex(gs, Wh, Hh, sh, MAX_DEPTH, i, hr, None, **kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        res[f"ms_hrls_{name}"] = round(ms, 4)
        log(f"[bench] layers {name}: HRLS render {ms:.3f} ms")
    res["overhead"] = round(res["ms_hrls_layers"] / res["ms_hrls_plain"] - 1.0, 4)
    return res


def spp_pairs_block(log, steps=8, batch=8):
    """The paper's training iteration with a random spp pair per iteration (Sec. 4):
    the paper's x4 network, robust loss, SGD; every iteration renders its batch of
    128x128 windows (HRLS at spp_h, LRHS at spp_l, drawn from the paper's sets) and
    takes one step.  Two procedural training scenes, 4 windows each."""
    import numpy as np
    import torch
    import paper_2106_12802_amd as mrs
    from paper_2106_12802_amd import hybrid as Hy
    data = Hy.OnlinePairs([(100, 20000), (101, 60000)], windows=4, size=128, log=None)
    net = mrs.FusionNet(seed=1, arch="rdg")
    Hy.train_random_spp(net, data, 1, batch=batch, log=None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = Hy.train_random_spp(net, data, steps, batch=batch, seed=1, log=None)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    paths = [batch * 128 * 128 * (h + l / 16) for _, h, l, _ in hist]
    net.close()
    data.close()
    res = {"workload": f"paper network x4, robust loss, SGD; batch {batch} of 128x128 windows "
                       "from 2 procedural scenes (20k, 60k triangles), inputs rendered every "
                       "iteration at a random spp pair",
           "ms_per_iteration": round(ms, 3),
           "spp_pairs": [[h, l] for _, h, l, _ in hist],
           "mpaths_per_iteration_mean": round(float(np.mean(paths)) / 1e6, 3)}
    log(f"[bench] random spp pairs: {ms:.2f} ms per iteration ({res['spp_pairs']})")
    if os.path.exists(WEIGHTS):
        res["spp_sweep"] = spp_sweep(log)
    return res


def spp_sweep(log):
    """The paper's spp-pair table (Table 6) on the bench scene at 1280x720: PSNR of the
    hybrid frame for HRLS {1, 2, 4, 8} x LRHS {16, 64, 256} spp with the trained trunk
    (and with a trunk trained on random spp pairs, when such weights are present)."""
    import paper_2106_12802_amd as mrs
    from mrs_inputs import scenes as S
    from paper_2106_12802_amd import hybrid as HY
    gs = mrs.GpuScene(S.procedural(SCENE_SEED))
    W, H = HRLS[0], HRLS[1]
    ref = HY.reference(gs, W, H, 1024, HY.REF_SEED)
    out = {"reference": "1280x720 at 1024 spp, FP64 pixel sums, independent seed"}
    nets = [("fixed_4_64", WEIGHTS)]
    if os.path.exists(WEIGHTS_RSPP):
        nets.append(("random_spp", WEIGHTS_RSPP))
    for name, path in nets:
        net = mrs.FusionNet()
        net.load_weights(path)
        table = HY.spp_grid(gs, net, W, H, ref=ref)
        net.close()
        out[name] = {f"{h}/{l}": round(p, 2) for (h, l), p in sorted(table.items())}
        out[name + "_monotone"] = HY.grid_monotone(table)
        log(f"[bench] spp sweep {name}: {out[name]} monotone {out[name + '_monotone']}")
    gs.close()
    return out


ABLATIONS_JSON = os.path.join(ROOT, "paper_2106_12802_amd", "weights", "ablations.json")


def ablations_block(log, scenes=((7, None), (200, None))):
    """The trained ablation networks (paper_2106_12802_amd/weights/ablations.json):
    with and without the HRLS render layers as inputs, and the paper's network
    trained with its own recipe (robust loss, SGD) against L1 with the same
    optimiser: each network's hybrid 720p frame PSNR against an independent
    1024-spp reference, on the bench scene and a held-out scene, plus the
    record of its training run."""
    import torch
    import paper_2106_12802_amd as mrs
    from paper_2106_12802_amd import hybrid
    from paper_2106_12802_amd.metrics import image_metrics
    from mrs_inputs import scenes as S
    if not os.path.exists(ABLATIONS_JSON):
        return None
    meta = json.load(open(ABLATIONS_JSON))
    wdir = os.path.dirname(ABLATIONS_JSON)
    specs = dict(S.training_scene_specs(200, 1))
    evals = []
    for seed, _ in scenes:
        scene = S.procedural(seed) if seed == 7 else S.procedural_sized(seed, specs[seed])
        gs = mrs.GpuScene(scene)
        evals.append((f"bench" if seed == 7 else f"heldout_{seed}", gs,
                      hybrid.reference(gs, 1280, 720, 1024, hybrid.REF_SEED + seed)))
    out = {}
    for study, rec in meta.items():
        res = {"training": rec.get("training"), "psnr_at_training": rec.get("psnr_at_training")}
        for arch_key, fname in rec["weights"].items():
            path = os.path.join(wdir, fname)
            if not os.path.exists(path):
                continue
            arch = rec.get("arch", {}).get(arch_key, arch_key)
            net = mrs.FusionNet(arch=arch)
            net.load_weights(path)
            r = {}
            for k, (name, gs, ref) in enumerate(evals):
                img, _ = hybrid.hybrid_frame(gs, net, 1280, 720, 1000 + k)
                torch.cuda.synchronize()
                r[name] = round(image_metrics(img, ref)["psnr"], 3)
            net.close()
            res[arch_key] = r
            log(f"[bench] ablation {study} {arch_key}: {r}")
        out[study] = res
    for _, gs, _ in evals:
        gs.close()
    return out


def res16_flop(B, H, W):
    """Forward FLOP of the 16-residual-block network on B frames of H x W (x4):
    2 x sum over convs of output pixels x C_out x C_in x k^2."""
    hr, lr = B * H * W, B * H * W // 16
    mac = (hr * 64 * 10 * 9 + lr * 64 * 3 * 9 + lr * 64 * 1088 + 32 * lr * 64 * 64 * 9
           + lr * 256 * 64 * 9 + hr * 3 * 80 * 9)
    return 2 * mac


def training_block(log, steps=20, warmup=5):
    """The configured training step (16-residual-block network, batch 16 of 128 x 128
    HR / 32 x 32 LR crops, L1 loss reduced in FP64, Adam at lr 1e-4, BF16 MFMA with
    FP32 masters): ms per step and the MFMA rate it reaches.  One step is the
    forward, the data gradients of every conv but the two input convs, every
    weight gradient (each as many FLOP as its forward conv) and the update."""
    import torch
    import paper_2106_12802_amd as mrs
    B, H, W = 16, 128, 128
    g = torch.Generator(device="cuda").manual_seed(11)
    hr = torch.rand(B, H, W, 3, device="cuda", generator=g) * 2.0
    aux = torch.rand(B, H, W, 7, device="cuda", generator=g)
    lr = torch.rand(B, H // 4, W // 4, 3, device="cuda", generator=g) * 2.0
    tgt = torch.rand(B, H, W, 3, device="cuda", generator=g) * 2.0
    net = mrs.FusionNet(seed=3)
    for _ in range(warmup):
        net.train_step(hr, aux, lr, tgt, lr=1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        net.train_step(hr, aux, lr, tgt, lr=1e-4)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    fwd = res16_flop(B, H, W)
    in_convs = 2 * (B * H * W * 64 * 10 * 9 + B * H * W // 16 * 64 * 3 * 9)
    flop = 3 * fwd - in_convs
    loss = net.train_step(hr, aux, lr, tgt, lr=1e-4, want_loss=True)
    net.close()
    res = {"workload": "16-residual-block network, batch 16 of 128x128 HR / 32x32 LR crops, "
                       "L1 (FP64 reduction) + Adam lr 1e-4, BF16 MFMA with FP32 masters",
           "ms_per_step": round(ms, 3), "gflop_per_step": round(flop / 1e9, 2),
           "tflops": round(flop / (ms / 1e3) / 1e12, 2),
           "frac_of_bf16_peak": round(flop / (ms / 1e3) / 1e12 / PEAK_BF16_TFLOPS, 5),
           "loss_after_steps": round(float(loss), 5)}
    log(f"[bench] training step (cfg of 16 x 128^2): {ms:.3f} ms, {res['tflops']} TFLOP/s")
    return res


def paper_net_block(log, reps=10, train_steps=10):
    """The paper's own network (three residual dense groups, Sec. 4): fuse time
    on the 720p hybrid frame and at the paper's runtime-table size (one
    1024 x 1024 image, x4), and the training step (batch 16 of 128 x 128 HR
    crops, robust loss, SGD) -- random weights and inputs of those shapes."""
    import torch
    import paper_2106_12802_amd as mrs
    g = torch.Generator(device="cuda").manual_seed(5)
    res = {}
    for arch, sc in (("rdg", 4), ("rdg_x2", 2), ("rdg_x8", 8)):
        net = mrs.FusionNet(seed=1, arch=arch)
        sizes = (("720p", (720, 1280)), ("1024x1024", (1024, 1024)))
        for tag, (H, W) in sizes if sc == 4 else sizes[1:]:
            hr = torch.rand(H, W, 3, device="cuda", generator=g)
            aux = torch.rand(H, W, 7, device="cuda", generator=g)
            lr = torch.rand(H // sc, W // sc, 3, device="cuda", generator=g)
            out = torch.empty_like(hr)
            net.fuse(hr, aux, lr, out=out)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                net.fuse(hr, aux, lr, out=out)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / reps
            flop = rdg_flop(H, W, sc)
            key = f"x{sc}_{tag}"
            res[f"fuse_ms_{key}"] = round(ms, 4)
            res[f"tflops_{key}"] = round(flop / (ms / 1e3) / 1e12, 2)
            log(f"[bench] paper network x{sc} {tag}: {ms:.3f} ms ({flop / 1e9:.1f} GFLOP)")
        res[f"params_x{sc}"] = net.num_params
        res[f"paper_table5_x{sc}_1024sq_ms"] = PAPER_TABLE5_S[sc] * 1e3
        if sc != 4:
            net.close()
        else:
            keep = net
    net = keep
    res["gflop_x4_720p"] = round(rdg_flop(720, 1280) / 1e9, 2)
    res["frac_x4_720p"] = round(res["tflops_x4_720p"] / PEAK_BF16_TFLOPS, 5)
    B, H, W = 16, 128, 128
    t = [torch.rand(B, H, W, c, device="cuda", generator=g) for c in (3, 7)]
    t.insert(2, torch.rand(B, H // 4, W // 4, 3, device="cuda", generator=g))
    t.append(torch.rand(B, H, W, 3, device="cuda", generator=g))
    net.train_step(*t, lr=1e-4, loss="robust", beta=0.1, optimizer="sgd")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(train_steps):
        net.train_step(*t, lr=1e-4, loss="robust", beta=0.1, optimizer="sgd")
    torch.cuda.synchronize()
    res["train_step_ms_b16_128"] = round((time.perf_counter() - t0) * 1e3 / train_steps, 3)
    log(f"[bench] paper network training step: {res['train_step_ms_b16_128']} ms")
    net.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--equal-psnr-scenes", type=int, default=3,
                    help="held-out scenes in the equal-PSNR comparison (0: skip it)")
    ap.add_argument("--batch-scenes", type=int, default=32,
                    help="scenes in the batched render+fuse measurement (0: skip it)")
    ap.add_argument("--no-two-calls", action="store_true",
                    help="skip the comparison runs (one frame at a time, two separate render "
                         "calls) and the per-kernel breakdown pass (profiling runs: every "
                         "k_extend launch is then one of the timed kind)")
    ap.add_argument("--no-mis", action="store_true",
                    help="skip the multiple-importance-sampling comparison")
    ap.add_argument("--no-camera", action="store_true",
                    help="skip the depth-of-field / motion-blur and render-layer timing blocks")
    ap.add_argument("--no-spp-pairs", action="store_true",
                    help="skip the random-spp-pair training iteration block")
    ap.add_argument("--no-paper-net", action="store_true",
                    help="skip timing the paper's own network (residual dense groups)")
    ap.add_argument("--no-training", action="store_true",
                    help="skip timing the training step of the 16-residual-block network")
    ap.add_argument("--no-ablations", action="store_true",
                    help="skip evaluating the trained ablation networks (input layers, loss)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 1 GiB device copy first (PMC byte-counter calibration)")
    ap.add_argument("--chunk-paths", type=int, default=None, help="tuning: paths resident at once")
    ap.add_argument("--trace-blocks", type=int, default=None, help="tuning: traversal grid size")
    ap.add_argument("--schedule", type=int, default=None, choices=(0, 1),
                    help="tuning: traversal queue schedule (0 grid-stride, 1 dynamic)")
    ap.add_argument("--streams", type=int, default=None,
                    help="tuning: concurrent sub-chunks per render (1..4)")
    ap.add_argument("--tail-bounce", type=int, default=None,
                    help="tuning: first bounce traced path by path in one launch (65: never)")
    ap.add_argument("--bvh-quantized", type=int, default=None, choices=(0, 1),
                    help="tuning: traverse the quantized 64-byte BVH4 nodes")
    ap.add_argument("--queue-sort", type=int, default=None, choices=(0, 1),
                    help="tuning: order appended rays by octant / shadow rays by light")
    ap.add_argument("--conv-small-tiles", type=int, default=None,
                    help="tuning: 3x3 convs with fewer 16x16 output tiles run the small-tile plan")
    ap.add_argument("--net-fused-blocks", type=int, default=None, choices=(0, 1),
                    help="tuning: the network trunk's residual blocks as one kernel each")
    ap.add_argument("--frames-in-flight", type=int, default=2, choices=(1, 2),
                    help="frames the timed frame stream keeps in flight")
    ap.add_argument("--wave-extend", type=int, default=None,
                    help="tuning: bounces below this trace closest-hit rays a wave at a time")
    ap.add_argument("--wave-shadow", type=int, default=None,
                    help="tuning: bounces below this trace shadow rays a wave at a time")
    ap.add_argument("--bvh-builder", default=None, choices=("lbvh", "ploc"),
                    help="tuning: BVH builder of the scenes (default ploc)")
    ap.add_argument("--leaf-max", type=int, default=None,
                    help="BVH build: triangles a BVH4 leaf may group (1..4)")
    ap.add_argument("--stats-summary", metavar="PROF_DIR",
                    help="summarise a rocprofv3 --stats run into the profiles/ kernel-stats file")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="summarise two rocprofv3 --pmc runs into the profiles/ traffic file")
    ap.add_argument("--counters-summary", nargs=3, metavar=("VALU_DIR", "CACHE_DIR", "MFMA_DIR"),
                    help="summarise the three rocprofv3 --pmc counter passes into profiles/")
    args = ap.parse_args()
    if args.counters_summary:
        counters_summary(args.counters_summary, COUNTERS_SUMMARY)
        return
    if args.stats_summary:
        stats_summary(args.stats_summary, STATS_SUMMARY)
        return
    if args.pmc_summary:
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], TRAFFIC_SUMMARY)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU path is a design, not part of this build)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2106_12802_amd as mrs
    from paper_2106_12802_amd import hybrid as HY
    from paper_2106_12802_amd import tracer as R
    from mrs_inputs import scenes as S

    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration()
    R.set_tuning(args.chunk_paths, args.trace_blocks, args.schedule, args.leaf_max, args.streams,
                 args.tail_bounce, args.bvh_builder, queue_sort=args.queue_sort,
                 bvh_quantized=args.bvh_quantized, wave_extend=args.wave_extend,
                 wave_shadow=args.wave_shadow, conv_small_tiles=args.conv_small_tiles,
                 net_fused_blocks=args.net_fused_blocks)
    tuning = R.get_tuning()
    log(f"[bench] tuning {tuning}")
    scene = S.procedural(SCENE_SEED)
    gs = mrs.GpuScene(scene)
    net = mrs.FusionNet()
    trained = os.path.exists(WEIGHTS)
    if trained:
        net.load_weights(WEIGHTS)
    else:
        net.init(1)
    torch.cuda.synchronize()
    (Wh, Hh, sh), (Wl, Hl, sl) = HRLS, LRHS
    hr_rgb = torch.empty(Hh, Wh, 3, device="cuda")
    hr_aux = torch.empty(Hh, Wh, 7, device="cuda")
    lr_rgb = torch.empty(Hl, Wl, 3, device="cuda")
    out = torch.empty(Hh, Wh, 3, device="cuda")
    paths = Wh * Hh * sh + Wl * Hl * sl

    # HRLS and LRHS go through the wavefront together as one two-job batch
    # (one launch sequence over both renders); each frame gets new seeds
    frame_batch = mrs.Batch([
        dict(scene=gs, W=Wh, H=Hh, spp=sh, max_depth=MAX_DEPTH, seed=0, out_rgb=hr_rgb,
             out_aux=hr_aux),
        dict(scene=gs, W=Wl, H=Hl, spp=sl, max_depth=MAX_DEPTH, seed=1, out_rgb=lr_rgb,
             want_aux=False)])

    def step(i):
        frame_batch.set_seeds([2 * i, 2 * i + 1])
        frame_batch.render()
        net.fuse(hr_rgb, hr_aux, lr_rgb, out=out)

    # a second frame in flight: its own batch (path workspace) and images
    hr_rgb2, hr_aux2 = torch.empty_like(hr_rgb), torch.empty_like(hr_aux)
    lr_rgb2 = torch.empty_like(lr_rgb)
    frame_batch2 = mrs.Batch([
        dict(scene=gs, W=Wh, H=Hh, spp=sh, max_depth=MAX_DEPTH, seed=0, out_rgb=hr_rgb2,
             out_aux=hr_aux2),
        dict(scene=gs, W=Wl, H=Hl, spp=sl, max_depth=MAX_DEPTH, seed=1, out_rgb=lr_rgb2,
             want_aux=False)])
    in_flight = ([frame_batch, frame_batch2], [
        lambda: net.fuse(hr_rgb, hr_aux, lr_rgb, out=out),
        lambda: net.fuse(hr_rgb2, hr_aux2, lr_rgb2, out=out)])

    def frames(first, k, n=args.frames_in_flight):
        # k frames pipelined on the stream, n in flight: frame i+1 renders while
        # frame i's last paths finish and while frame i is fused
        HY.pipeline_frames(in_flight[0][:n], lambda i: [2 * i, 2 * i + 1], in_flight[1][:n],
                           range(first, first + k))

    def step_calls(i):
        R.render_ex(gs, Wh, Hh, sh, MAX_DEPTH, 2 * i, hr_rgb, hr_aux)
        R.render_ex(gs, Wl, Hl, sl, MAX_DEPTH, 2 * i + 1, lr_rgb, None)
        net.fuse(hr_rgb, hr_aux, lr_rgb, out=out)

    # algorithmic work of one frame (counting variant of the traversal kernels)
    R.counters(reset=True)
    R.set_count_work(True)
    step(0)
    R.set_count_work(False)
    work = R.counters(reset=True)
    log(f"[bench] work per frame: {json.dumps(work)}")

    if args.warmup:
        frames(0, args.warmup)
    torch.cuda.synchronize()
    log(f"[bench] warmup done ({args.warmup} frames)")

    # timed frames, pipelined: HIP events around the roofline kernel's launches only
    R.profile_select(["extend"])
    R.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    frames(0, args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof_ext = R.profile_read()
    R.profile_enable(False)
    R.profile_select(None)
    ms_per_step = dt * 1e3 / args.steps
    value = paths * args.steps / dt / 1e6
    log(f"[bench] {args.steps} frames: {ms_per_step:.3f} ms/frame, {value:.1f} Mpaths/s")
    # the same frames one at a time with every kernel's events, for the
    # per-kernel breakdown (not timed; skipped with the comparison runs, so that a
    # profiled run holds only the timed kind of launch)
    prof = prof_ext
    if not args.no_two_calls:
        R.profile_enable(True)
        for i in range(args.steps):
            step(i)
        prof = R.profile_read()
        R.profile_enable(False)
    # the same frames one at a time (each frame's fusion after its render), no
    # events: the latency of one frame, for comparison
    ms_unpiped = None
    if not args.no_two_calls:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for i in range(args.steps):
            step(i)
        torch.cuda.synchronize()
        ms_unpiped = (time.perf_counter() - t1) * 1e3 / args.steps
        log(f"[bench] same frames one at a time: {ms_unpiped:.3f} ms/frame")
    # the same frames as two separate render calls (for comparison, not timed above)
    ms_calls = None
    if not args.no_two_calls:
        step_calls(0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for i in range(args.steps):
            step_calls(i)
        torch.cuda.synchronize()
        ms_calls = (time.perf_counter() - t1) * 1e3 / args.steps
        log(f"[bench] same frames as two render calls: {ms_calls:.3f} ms/frame")

    ext_ms, ext_n = prof_ext.get("extend", (0.0, 0))
    ext_rays = max(work["rays"] - work["tail_rays"], 1)  # rays traced by k_extend itself
    flop_frame = (FLOP_PER_VISIT * work["extend_visits"] + FLOP_PER_TEST * work["extend_tests"]
                  + FLOP_PER_RAY * ext_rays)
    launches_per_frame = ext_n / args.steps if args.steps else 0
    flop_per_launch = flop_frame / max(launches_per_frame, 1)
    avg_launch_s = ext_ms / 1e3 / max(ext_n, 1)
    achieved = flop_per_launch / avg_launch_s / 1e12 if avg_launch_s > 0 else 0.0
    roofline = {"bound": "alu", "kernel": "k_extend (closest-hit traversal)",
                "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 5), "traffic": read_traffic(),
                "avg_launch_us": round(avg_launch_s * 1e6, 2),
                "flop_per_launch": int(flop_per_launch),
                "visits_per_ray": round(work["extend_visits"] / ext_rays, 2),
                "tests_per_ray": round(work["extend_tests"] / ext_rays, 2)}
    # the network alone: in the pipelined frames it shares the GPU with the next
    # frame's render, so its events there also hold the tracer's share
    R.profile_enable(True)
    for _ in range(args.steps):
        net.fuse(hr_rgb, hr_aux, lr_rgb, out=out)
    torch.cuda.synchronize()
    prof_cnn = R.profile_read()
    R.profile_enable(False)
    cnn_ms = sum(prof_cnn.get(k, (0.0, 0))[0] for k in ("cnn_prep", "cnn_hr_in", "cnn_lr",
                                                         "cnn_hr_out")) / args.steps
    cnn_roof = {"bound": "mfma", "achieved": round(CNN_FLOP_720P / (cnn_ms / 1e3) / 1e12, 2)
                if cnn_ms > 0 else 0.0, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                "ms_per_frame": round(cnn_ms, 4), "measured": "the network alone, HIP events"}
    cnn_roof["frac"] = round(cnn_roof["achieved"] / PEAK_BF16_TFLOPS, 5)
    # hardware counters of the committed profile, if it belongs to these kernel sources
    ctr = read_counters()
    roofline["counters"] = None if ctr is None else {
        k: ctr[k] for k in ("k_extend_wave", "k_extend", "k_shadow", "k_tail") if k in ctr}
    cnn_roof["counters"] = None if ctr is None else {
        k: ctr[k] for k in ctr if k.startswith("k_conv") or k == "k_res_block"}
    kernel_ms = {k: round(v[0] / args.steps, 4) for k, v in prof.items()}
    result = {
        "metric": METRIC, "value": round(value, 3), "unit": "Mpaths/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+bf16",
        "data": "synthetic",
        "config": {"workload": "720p hybrid frame: procedural scene (seed 7, 101,446 triangles, "
                               "textured Lambert+GGX, 3 quad lights, env 0.2), HRLS 1280x720@4spp "
                               "+ LRHS 320x180@64spp (max depth 8, RR from vertex 3; both renders as one "
                               "two-job batch, new seeds every frame) + BF16 fusion network "
                               "(175.7 GFLOP); frames pipelined on one stream with "
                               f"{args.frames_in_flight} in flight (frame i+1 renders while frame i's "
                               "last paths finish and while frame i is fused)",
                   "paths_per_frame": paths, "triangles": scene.num_tris,
                   "weights": "trained (paper_2106_12802_amd/weights)" if trained else "untrained",
                   "tuning": tuning},
        "roofline": roofline,
        "roofline_cnn": cnn_roof,
        "kernel_ms_per_frame": kernel_ms,
        "rays_per_path": round((work["rays"] + work["shadow_rays"]) / paths, 3),
        "ms_per_frame_unpipelined": None if ms_unpiped is None else round(ms_unpiped, 4),
        "ms_per_frame_two_render_calls": None if ms_calls is None else round(ms_calls, 4),
    }
    if args.equal_psnr_scenes > 0:
        result["equal_psnr"] = equal_psnr_block(net, args.equal_psnr_scenes, log)
    if args.batch_scenes > 0:
        result["batched"] = batched_block(net, log, args.batch_scenes)
    if not args.no_training:
        result["training"] = training_block(log)
    if not args.no_ablations:
        result["ablations"] = ablations_block(log)
    if not args.no_paper_net:
        result["paper_net"] = paper_net_block(log)
    if not args.no_mis:
        result["mis"] = mis_block(gs, log)
    if not args.no_camera:
        result["camera"] = camera_block(gs, log)
        result["layers"] = layers_block(gs, log)
    if not args.no_spp_pairs:
        result["spp_pairs"] = spp_pairs_block(log)
    if not args.no_cpu_baseline:
        # every CPU this process may run on, at most the 16 that a one-GPU machine grants
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        log(f"[bench] timing the FP64 oracle on {threads} host threads (nproc "
            f"{os.cpu_count()}, affinity {len(os.sched_getaffinity(0))})")
        result["cpu_baseline"] = cpu_baseline(scene, threads)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
