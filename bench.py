"""Benchmark: one step = the whole hot path on one MI355X -- LEB build of an
adaptive conforming tet grid from a 256^3 fBm cloud density resident in HBM
(1-pixel camera target), then a 1024 x 1024, 32 spp, 32-bounce render of it.

Prints one JSON line.  `value` is Msamples/s of whole steps (build + render);
tet-steps/s, render-only and build figures are reported beside it, with the
render kernel's roofline fraction and the CPU oracle timed on a bounded
sample of the same workload.  The radiance-cache leg ("nrc") trains the
cache online on the same grid and compares, at equal RMSE against a
1024-spp plain render, the time of truncated renders with the cache (plus
one training frame each) with the plain renderer's.  The batch leg
("batch") renders 64 small scenes (64^2..512^2, 4..64 spp, 3k..5M tets) as
one captured HIP-graph frame and as 64 tet_render calls one after another.
The camera-path leg ("camera_path") rebuilds the grid for a moving camera
with leb_update and times it against scratch builds.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Msamples/s + tet-steps/s at 1024² 32spp; NRC vs plain speedup at equal RMSE"
HBM_PEAK_GBS = 8000.0
BYTES_PER_TET_STEP = 32  # algorithmic bytes per walk step (compact tet record)
MFMA_BF16_PEAK_TFLOPS = 2500.0  # dense BF16 matrix-core peak
NRC_FLOP_PER_QUERY = 2 * (76 * 64 + 3 * 64 * 64 + 64 * 3)  # multiply-adds of the 76-64-64-64-64-3 network
TRAFFIC_GLOB = os.path.join(ROOT, "profiles", "render_cloud1024*_traffic.txt")
PLUME_TRAFFIC_GLOB = os.path.join(ROOT, "profiles", "render_plume1024*_traffic.txt")
LAUNCH_KEYS = ("waves_per_simd", "event_wait", "batch_items", "block_size", "record_layout", "samples_per_item")
COPY_BYTES = 1 << 30  # plain device copy used to calibrate the traffic counters
KERNEL_SOURCES = ["paper_2506_11510_amd/csrc/render.hip", "paper_2506_11510_amd/csrc/common.h"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_kv(path):
    out = {}
    try:
        with open(path) as f:
            for line in f:
                if "=" in line and not line.startswith("#"):
                    k, v = line.split("=", 1)
                    out[k.strip()] = v.strip()
    except OSError:
        pass
    return out


def measured_traffic(launch: dict, pattern: str = TRAFFIC_GLOB):
    """HBM bytes per tracing-kernel launch from the committed rocprofv3
    counter runs of this launch configuration, or None when none was
    profiled or the kernel source changed since."""
    import glob
    want = {k: int(launch[k]) for k in LAUNCH_KEYS}
    for path in sorted(glob.glob(pattern)):
        t = read_kv(path)
        if t.get("source_hash") != kernel_source_hash() or "traffic_bytes_per_launch" not in t:
            continue
        try:
            got = json.loads(t.get("launch", "{}"))
        except ValueError:
            continue
        if {k: got.get(k) for k in LAUNCH_KEYS} == want:
            return float(t["traffic_bytes_per_launch"])
    return None


def traffic_fractions(traffic, algorithmic_bytes: float, kernel_ms: float) -> dict:
    """Counter traffic over the kernel time against the HBM peak, and the
    share of it the method needs (algorithmic / counted bytes)."""
    if not traffic:
        return {"frac_traffic": None, "line_utilisation": None}
    return {"frac_traffic": round(traffic / (kernel_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "line_utilisation": round(algorithmic_bytes / traffic, 4)}


def _counter_rows(d):
    import csv
    import glob
    rows = []
    for p in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        rows += list(csv.DictReader(open(p)))
    return rows


def tracing_part(kernel_name: str):
    """Which part of a plain render's tracing a dispatch is: "main" (the
    persistent tracing kernel), "light" (the queued light rays: their keys,
    sort and walks), or None."""
    if "k_render<" in kernel_name and ", 0, false, false>" in kernel_name:
        return "main"
    if "k_light" in kernel_name or "rocprim" in kernel_name:
        return "light"
    return None


def summarize_pmc(fetch_dir, write_dir, out_path, command, workload="the 1024^2 x 32 spp cloud frame"):
    """Traffic of the tracing from FETCH_SIZE / WRITE_SIZE runs (KiB per
    dispatch), each scaled by the factor that maps the same counter on a
    plain 1 GiB device copy to its true size; per launch of the tracing
    kernel, with the dispatches of its queued light rays."""
    def per_kernel(rows, counter):
        parts, copies = {"main": [], "light": []}, []
        for r in rows:
            if r["Counter_Name"] != counter:
                continue
            v = float(r["Counter_Value"])
            part = tracing_part(r["Kernel_Name"])
            if part:
                parts[part].append(v)
            elif "copyBuffer" in r["Kernel_Name"]:
                copies.append(v)
        return parts, copies
    fp, fc = per_kernel(_counter_rows(fetch_dir), "FETCH_SIZE")
    wp, wc = per_kernel(_counter_rows(write_dir), "WRITE_SIZE")
    ft, wt = fp["main"], wp["main"]
    f_kib = (sum(ft) + sum(fp["light"])) / len(ft)
    w_kib = (sum(wt) + sum(wp["light"])) / len(wt)
    f_fac = (COPY_BYTES / 1024) / max(fc)
    w_fac = (COPY_BYTES / 1024) / max(wc)
    traffic = (f_kib * f_fac + w_kib * w_fac) * 1024
    with open(out_path, "w") as f:
        f.write(f"# HBM traffic of the tracing kernel k_render<TetMedium32> on {workload}\n")
        f.write(f"# command: {command}\n")
        f.write("# counters are KiB per dispatch; the copy factors map a plain 1 GiB device copy to 1 GiB\n")
        f.write(f"source_hash = {kernel_source_hash()}\n")
        m = re.search(r"--launch '(\{[^']*\})'", command)
        if m:
            f.write(f"launch = {m.group(1)}\n")
        f.write(f"dispatches = {len(ft)}\n")
        f.write(f"fetch_kib_per_launch = {f_kib:.1f}\n")
        f.write(f"write_kib_per_launch = {w_kib:.1f}\n")
        f.write(f"fetch_kib_per_launch_light_rays = {sum(fp['light']) / len(ft):.1f}\n")
        f.write(f"write_kib_per_launch_light_rays = {sum(wp['light']) / len(wt):.1f}\n")
        f.write(f"copy_fetch_kib = {max(fc):.1f}\n")
        f.write(f"copy_write_kib = {max(wc):.1f}\n")
        f.write(f"copy_fetch_factor = {f_fac:.4f}\n")
        f.write(f"copy_write_factor = {w_fac:.4f}\n")
        f.write(f"traffic_bytes_per_launch = {traffic:.6g}\n")
    print(open(out_path).read())


def summarize_counters(pmc_dir, out_path, command, steps_per_launch: float = 0.0):
    """Every counter collected on the tracing, per launch of the tracing
    kernel (with the dispatches of its queued light rays), with the L2 hit
    rate and VALU instructions per tet step."""
    rows = [r for r in _counter_rows(pmc_dir) if tracing_part(r["Kernel_Name"])]
    acc, cnt = {}, {}
    for r in rows:
        k = r["Counter_Name"]
        acc[k] = acc.get(k, 0.0) + float(r["Counter_Value"])
        if tracing_part(r["Kernel_Name"]) == "main":
            cnt[k] = cnt.get(k, 0) + 1
    avg = {k: acc[k] / cnt[k] for k in acc if cnt.get(k)}
    with open(out_path, "w") as f:
        f.write("# rocprofv3 counters of the tracing (k_render<TetMedium32> and the walks of its queued light rays),"
                " per launch\n")
        f.write(f"# command: {command}\n")
        f.write(f"source_hash = {kernel_source_hash()}\n")
        m = re.search(r"--launch '(\{[^']*\})'", command)
        if m:
            f.write(f"launch = {m.group(1)}\n")
        f.write(f"dispatches = {max(cnt.values()) if cnt else 0}\n")
        for k in sorted(avg):
            f.write(f"{k} = {avg[k]:.6g}\n")
        hit, miss = avg.get("TCC_HIT_sum"), avg.get("TCC_MISS_sum")
        if hit is not None and miss is not None and hit + miss > 0:
            f.write(f"l2_hit_rate = {hit / (hit + miss):.4f}\n")
        if steps_per_launch and "SQ_INSTS_VALU" in avg:
            f.write(f"tet_steps_per_launch = {steps_per_launch:.6g}\n")
            f.write(f"valu_wave_instructions_per_tet_step = {avg['SQ_INSTS_VALU'] / steps_per_launch:.4f}\n")
            f.write(f"valu_issue_slots_per_tet_step = {64 * avg['SQ_INSTS_VALU'] / steps_per_launch:.2f}\n")
    print(open(out_path).read())


def summarize_trace(trace_dir, out_path, command):
    """Short kernel table from a rocprofv3 --kernel-trace --stats run."""
    import csv
    import glob
    paths = glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)
    rows = list(csv.DictReader(open(paths[0])))
    with open(out_path, "w") as f:
        f.write(f"# rocprofv3 kernel statistics\n# command: {command}\n")
        f.write(f"{'calls':>6} {'avg_us':>12} {'total_ms':>10} {'pct':>6}  kernel\n")
        for r in rows[:16]:
            f.write(f"{int(r['Calls']):>6} {float(r['AverageNs']) / 1e3:>12.1f} {float(r['TotalDurationNs']) / 1e6:>10.2f} "
                    f"{float(r['Percentage']):>6.2f}  {r['Name'][:110]}\n")
        main = [r for r in rows if tracing_part(r["Name"]) == "main"]
        light = [r for r in rows if tracing_part(r["Name"]) == "light"]
        if main:
            launches = sum(int(r["Calls"]) for r in main)
            t_main = sum(float(r["TotalDurationNs"]) for r in main) / 1e6
            t_light = sum(float(r["TotalDurationNs"]) for r in light) / 1e6
            f.write(f"tracing_launches = {launches}\n")
            f.write(f"tracing_kernel_ms_per_launch = {t_main / launches:.3f}\n")
            f.write(f"queued_light_rays_ms_per_launch = {t_light / launches:.3f}  (keys, sort, walks)\n")
            f.write(f"tracing_ms_per_launch = {(t_main + t_light) / launches:.3f}\n")
    print(open(out_path).read())


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def cpu_baseline(sc, d, n_threads: int) -> dict:
    """The oracle, as it stands, on a bounded sample of the step: its full
    LEB build (its build is one thread) and a strided subset of the image's
    pixels at full spp, on `n_threads` OpenMP threads and on one thread; the
    render times are scaled to the full image."""
    import numpy as np
    import oracle
    cam = sc["camera"]
    t0 = time.perf_counter()
    g = oracle.leb_build(d, sc["n"], cam, sc["build"])
    t_build = time.perf_counter() - t0
    W, H = cam["width"], cam["height"]
    spp = sc["render"]["spp"]
    samples = W * H * spp

    def render_subset(stride, threads):
        pix = np.arange(0, W * H, stride, dtype=np.int32)
        t0 = time.perf_counter()
        _, st = g.render(cam, sc["medium"], sc["light"], spp, 2024, sc["render"], pixels=pix, threads=threads)
        t = time.perf_counter() - t0
        return len(pix), t, t * (W * H) / len(pix), st["tet_steps"]

    npx, t_render, t_full, steps = render_subset(3, n_threads)
    npx1, t_render1, t_full1, steps1 = render_subset(96, 1)
    return {"value": samples / (t_build + t_full) / 1e6, "unit": "Msamples/s", "cores": n_threads,
            "kind": "oracle",
            "sample": (f"oracle LEB build of the full grid ({g.num_tets} tets, 1 thread, {t_build:.1f} s) + render "
                       f"of every 3rd pixel ({npx} px x {spp} spp, {n_threads} threads, {t_render:.1f} s, "
                       f"{steps} tet steps) scaled to {W}x{H}"),
            "host": cpu_model(), "nproc": os.cpu_count(),
            "build_s": t_build, "render_s_full_image": t_full,
            "tet_steps_per_s": steps / t_render,
            "single_thread": {"value": samples / (t_build + t_full1) / 1e6, "unit": "Msamples/s",
                              "sample": f"every 96th pixel ({npx1} px x {spp} spp, 1 thread, {t_render1:.1f} s)",
                              "render_s_full_image": t_full1, "tet_steps_per_s": steps1 / t_render1}}


def dda_leg(tv, dev, sc, steps: int = 3) -> dict:
    """The regular-grid reference renderer (Amanatides-Woo over the same
    voxels, same integrator) on the benchmark frame."""
    cam, spp = sc["camera"], sc["render"]["spp"]
    ro = dict(sc["render"], samples_per_item=1, batch_items=64, waves_per_simd=5, event_wait=48)
    tv.dda_render(dev, sc["n"], 1.0, cam, sc["medium"], sc["light"], spp, 3, ro)
    ms, st = [], None
    for i in range(steps):
        _, st = tv.dda_render(dev, sc["n"], 1.0, cam, sc["medium"], sc["light"], spp, 30 + i, ro)
        ms.append(st["ms"])
    m = sum(ms) / len(ms)
    samples = cam["width"] * cam["height"] * spp
    return {"ms": round(m, 3), "msamples_per_s": round(samples / (m / 1e3) / 1e6, 3),
            "voxel_steps_per_frame": int(st["tet_steps"]),
            "voxel_steps_per_s": round(st["tet_steps"] / (st["trace_ms"] / 1e3), 1)}


def channels_leg(tv, torch, grid, sc, plain_ms: float, steps: int = 3) -> dict:
    """Extra per-tet channels on the benchmark frame: temperature, albedo
    and phase g grids at the density's resolution (seeded blobs), reduced
    to per-tet box means on the device, then the frame rendered with
    emission at real collisions and per-tet albedo and g."""
    cam, spp = sc["camera"], sc["render"]["spp"]
    import numpy as np
    import synthetic
    ch = {k: torch.from_numpy(v).cuda() for k, v in synthetic.channels(7, sc["n"]).items()}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    grid.set_channels(sc["n"], **ch)
    torch.cuda.synchronize()
    set_ms = (time.perf_counter() - t0) * 1e3
    ro = dict(sc["render"], channels=1, emission=[0.6, 0.35, 0.15])
    tv.render(grid, cam, sc["medium"], sc["light"], spp, 3, ro)
    ms, trace, st = [], [], None
    for i in range(steps):
        _, st = tv.render(grid, cam, sc["medium"], sc["light"], spp, 40 + i, ro)
        ms.append(st["ms"])
        trace.append(st["trace_ms"])
    m = float(np.mean(ms))
    samples = cam["width"] * cam["height"] * spp
    return {"channels": "temperature, albedo, g (%d^3 each)" % sc["n"], "set_channels_ms": round(set_ms, 3),
            "ms": round(m, 3), "trace_ms": round(float(np.mean(trace)), 3),
            "msamples_per_s": round(samples / (m / 1e3) / 1e6, 3), "overhead_vs_plain": round(m / plain_ms, 3),
            "tet_steps_per_frame": int(st["tet_steps"]), "real_collisions": int(st["real_collisions"])}


def density_model_leg(tv, torch, dev, sc, plain_ms: float, steps: int = 3) -> dict:
    """Density models inside the tets on the benchmark frame: linear between
    trilinear vertex samples (analytic light transmittance, as the plain
    frame, and ratio-tracked) and voxel lookup (ratio-tracked light), on a
    fresh grid of the same build; the voxel model is set beside the
    regular-grid tracer with the same light estimator (equal in
    expectation: image RMSE against it next to the RMSE between two
    regular-grid renders)."""
    import numpy as np
    cam, spp = sc["camera"], sc["render"]["spp"]
    scale = sc["build"]["density_scale"]
    g = tv.leb_build(dev, sc["n"], cam, build=sc["build"])
    out = {}
    imgs = {}
    for name, model, trans in (("linear", 1, 0), ("linear_ratio_light", 1, 1), ("voxel", 2, 1)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.set_density_model(model, dev, sc["n"], scale)
        torch.cuda.synchronize()
        set_ms = (time.perf_counter() - t0) * 1e3
        ro = dict(sc["render"], transmittance=trans)
        tv.render(g, cam, sc["medium"], sc["light"], spp, 3, ro)
        ms, trace, st = [], [], None
        for i in range(steps):
            img, st = tv.render(g, cam, sc["medium"], sc["light"], spp, 50 + i, ro)
            ms.append(st["ms"])
            trace.append(st["trace_ms"])
        imgs[name] = img.cpu().numpy()
        m = float(np.mean(ms))
        out[name] = {"transmittance": ["analytic", "ratio tracking"][trans], "set_model_ms": round(set_ms, 3),
                     "ms": round(m, 3), "trace_ms": round(float(np.mean(trace)), 3),
                     "msamples_per_s": round(cam["width"] * cam["height"] * spp / (m / 1e3) / 1e6, 3),
                     "vs_plain_ms": round(m / plain_ms, 3), "tet_steps_per_frame": int(st["tet_steps"]),
                     "null_collisions": int(st["null_collisions"]), "real_collisions": int(st["real_collisions"])}
    ro = dict(sc["render"], transmittance=1)
    d1, sd = tv.dda_render(dev, sc["n"], scale, cam, sc["medium"], sc["light"], spp, 60, ro)
    d2, _ = tv.dda_render(dev, sc["n"], scale, cam, sc["medium"], sc["light"], spp, 61, ro)
    d1, d2 = d1.cpu().numpy(), d2.cpu().numpy()
    out["voxel_vs_regular_grid"] = {
        "image_mean_tet_voxel": float(imgs["voxel"].mean()), "image_mean_regular_grid": float(d1.mean()),
        "rmse_tet_voxel_vs_regular_grid": float(np.sqrt(((imgs["voxel"] - d1) ** 2).mean())),
        "rmse_regular_grid_two_seeds": float(np.sqrt(((d2 - d1) ** 2).mean())),
        "regular_grid_ms": round(sd["ms"], 3)}
    del g
    return out


def sparse_build_leg(tv, torch, dev, sc, dense_grid) -> dict:
    """The same build from the volume's 8^3 bricks (OpenVDB-like leaves
    holding a nonzero voxel, extracted on the device): time, input and
    pyramid sizes against the dense build, and whether the grid is the
    dense build's (ids and neighbour links compared on the device)."""
    n = sc["n"]
    nb = n // 8
    v = dev.view(nb, 8, nb, 8, nb, 8).permute(0, 2, 4, 1, 3, 5).reshape(nb ** 3, 512)
    pick = torch.nonzero(v.ne(0).any(dim=1)).flatten()
    values = v.index_select(0, pick).contiguous()
    del v
    coords = torch.stack([pick % nb, (pick // nb) % nb, pick // (nb * nb)], dim=1).to(torch.int32).contiguous()
    ms = []
    for _ in range(2):
        g = tv.leb_build_sparse(coords, values, n, sc["camera"], build=sc["build"])
        ms.append(g.info()["ms"])
    a, b = g.export(device=True, fields=("ids", "nbr")), dense_grid.export(device=True, fields=("ids", "nbr"))
    same = bool(torch.equal(a["ids"], b["ids"]) and torch.equal(a["nbr"], b["nbr"]))
    nbr = int(pick.numel())
    dense_pyr = sum(((n >> l) ** 3) * 16 for l in range(1, 11) if (n >> l) > 0)
    sparse_pyr = nbr * 72 * 16 + sum(((n >> l) ** 3) * 16 for l in range(3, 11) if (n >> l) > 0) + nb ** 3 * 4
    del g, a, b, values, coords
    return {"bricks": nbr, "brick_positions": nb ** 3, "input_bytes": nbr * (512 * 4 + 12),
            "dense_input_bytes": n ** 3 * 4, "pyramid_bytes": sparse_pyr, "dense_pyramid_bytes": dense_pyr,
            "build_ms": round(ms[-1], 3), "same_grid_as_dense": same}


def camera_path_leg(tv, torch, dev, sc, frames: int = 16) -> dict:
    """The grid following a moving camera (the paper's real-time use):
    leb_update from the previous frame's grid against a scratch leb_build,
    per frame, on two scripted paths of the cloud: the benchmark camera
    orbiting 2 degrees and dollying 1 % a frame (the whole volume stays in
    view), and a close-up orbit 3 degrees a frame from 0.75 away, where the
    frustum clips the volume and the grid changes every frame.  Both grids
    are compared on the device every frame."""
    import numpy as np
    import synthetic
    out = {}
    close = dict(sc["camera"], pos=[0.5, 0.47, -0.25], look_at=[0.5, 0.5, 0.5])
    for name, cams in (("orbit", synthetic.camera_path(sc["camera"], frames + 1, 2.0, 0.01)),
                       ("close_up_orbit", synthetic.camera_path(close, frames + 1, 3.0, 0.0))):
        g = tv.leb_build(dev, sc["n"], cams[0], build=sc["build"])
        upd, scr, stood, same, tets = [], [], 0, True, []
        for cam in cams[1:]:
            g.update(dev, sc["n"], cam, build=sc["build"])
            r = tv.leb_build(dev, sc["n"], cam, build=sc["build"])
            a, b = g.info(), r.info()
            upd.append(a["ms"])
            scr.append(b["ms"])
            stood += a["rounds"] == 0
            tets.append(a["num_tets"])
            ea, eb = g.export(device=True, fields=("ids", "nbr")), r.export(device=True, fields=("ids", "nbr"))
            same = same and ea["ids"].shape == eb["ids"].shape and bool(torch.equal(ea["ids"], eb["ids"])) and \
                bool(torch.equal(ea["nbr"], eb["nbr"]))
            del r, ea, eb
        del g
        out[name] = {"frames": frames, "update_ms": round(float(np.mean(upd)), 3),
                     "scratch_build_ms": round(float(np.mean(scr)), 3),
                     "speedup": round(float(np.mean(scr)) / float(np.mean(upd)), 3),
                     "frames_tree_stood": int(stood), "tets_min_max": [int(min(tets)), int(max(tets))],
                     "same_grid_as_scratch_every_frame": same}
    return out


def regular_grid_1024_leg(tv, torch, dev, sc, steps: int = 2) -> dict:
    """The paper's comparison at its resolution: the cloud resampled to a
    1024^3 regular grid (trilinear, on the device), the adaptive tet grid
    built from that volume with the frame's settings, and both renderers on
    the frame (1024^2, 32 spp): the tet walk vs the voxel DDA over 1024^3."""
    import numpy as np
    n = 1024
    big = torch.nn.functional.interpolate(dev.view(1, 1, sc["n"], sc["n"], sc["n"]), size=(n, n, n),
                                          mode="trilinear", align_corners=False).reshape(-1).contiguous()
    cam, spp = sc["camera"], sc["render"]["spp"]
    g = tv.leb_build(big, n, cam, build=sc["build"])
    info = g.info()
    tv.render(g, cam, sc["medium"], sc["light"], spp, 3, sc["render"])
    tet = [tv.render(g, cam, sc["medium"], sc["light"], spp, 70 + i, sc["render"])[1]["ms"] for i in range(steps)]
    ro = dict(sc["render"], samples_per_item=1, batch_items=64, waves_per_simd=5, event_wait=48)
    tv.dda_render(big, n, 1.0, cam, sc["medium"], sc["light"], spp, 3, ro)
    dda = []
    for i in range(steps):
        _, st = tv.dda_render(big, n, 1.0, cam, sc["medium"], sc["light"], spp, 80 + i, ro)
        dda.append(st["ms"])
    del g, big
    t, d = float(np.mean(tet)), float(np.mean(dda))
    return {"volume": "cloud resampled to 1024^3", "num_tets": info["num_tets"], "build_ms": round(info["ms"], 3),
            "tet_render_ms": round(t, 3), "regular_grid_render_ms": round(d, 3),
            "regular_grid_voxel_steps": int(st["tet_steps"]), "tet_vs_regular_grid_speedup": round(d / t, 3),
            "cells_ratio": round(n ** 3 / info["num_tets"], 1)}


def host_io_leg(tv, torch, d, sc, steps: int = 3) -> dict:
    """The same step with host buffers at the boundary: the density read
    from host memory (uploaded over PCIe by the build) and the image
    written to host memory (copied back by the render)."""
    import numpy as np
    cam, spp = sc["camera"], sc["render"]["spp"]
    img = np.empty((cam["height"], cam["width"], 3), np.float32)
    g = tv.leb_build(d, sc["n"], cam, build=sc["build"])
    tv.render(g, cam, sc["medium"], sc["light"], spp, 5, sc["render"], out=img)
    del g
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        g = tv.leb_build(d, sc["n"], cam, build=sc["build"])
        tv.render(g, cam, sc["medium"], sc["light"], spp, 900 + i, sc["render"], out=img)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    return {"ms_per_step": round(ms, 3),
            "msamples_per_s": round(cam["width"] * cam["height"] * spp / (ms / 1e3) / 1e6, 3),
            "bytes_over_pcie_per_step": int(d.nbytes + img.nbytes)}


PLUME_LAUNCH = {"waves_per_simd": 5, "event_wait": 32, "batch_items": 64, "block_size": 256, "record_layout": 32,
                "samples_per_item": 1}


def plume_leg(tv, torch, host_rounds: bool = False, launch: dict | None = None) -> dict:
    """The production-scale configuration: 1024^3 plume density resident in
    HBM, adaptive LEB build (~86 M tets), 1024^2 renders at 32 and 1024 spp
    with 64 bounces.  Returns the figures and (grid, scene, 1024-spp image)
    for the radiance-cache leg."""
    import numpy as np
    import synthetic
    sc = synthetic.scene("plume")
    sc["render"] = dict(sc["render"], **(launch or PLUME_LAUNCH))
    if host_rounds:
        sc["build"] = dict(sc["build"], host_rounds=1)
    t0 = time.perf_counter()
    dev = torch.from_numpy(sc["density_fn"]()).cuda()
    gen_s = time.perf_counter() - t0
    builds = []
    for _ in range(2):
        g = tv.leb_build(dev, sc["n"], sc["camera"], build=sc["build"])
        builds.append(g.info())
    sparse = sparse_build_leg(tv, torch, dev, sc, g)
    del dev
    cam = sc["camera"]
    tv.render(g, cam, sc["medium"], sc["light"], 32, 1, sc["render"])
    r32 = []
    for i in range(3):
        _, st = tv.render(g, cam, sc["medium"], sc["light"], 32, 10 + i, sc["render"])
        r32.append(st)
    ref, st1024 = tv.render(g, cam, sc["medium"], sc["light"], 1024, 7777, sc["render"])
    ms32 = float(np.mean([r["ms"] for r in r32]))
    tr32 = float(np.mean([r["trace_ms"] for r in r32]))
    steps32 = float(np.mean([r["tet_steps"] for r in r32]))
    px = cam["width"] * cam["height"]
    achieved = steps32 * BYTES_PER_TET_STEP / (tr32 / 1e3) / 1e9
    traffic = measured_traffic(sc["render"], PLUME_TRAFFIC_GLOB)
    out = {"workload": "1024^3 curl-advected fBm plume (seed 2, 5% occupancy, sigma_t max 50) -> adaptive LEB grid "
                       "(1 px target, tau 0.2, depth <= 30) -> 1024x1024, 64 bounces, albedo 0.95, HG g 0.6",
           "density_gen_s_host": round(gen_s, 2), "num_tets": builds[-1]["num_tets"],
           "max_depth": builds[-1]["max_depth"], "build_rounds": builds[-1]["rounds"],
           "build_ms": round(builds[-1]["ms"], 3), "sparse_input": sparse,
           "spp32": {"ms": round(ms32, 3), "trace_ms": round(tr32, 3),
                     "msamples_per_s": round(px * 32 / (ms32 / 1e3) / 1e6, 3),
                     "tet_steps_per_s": round(steps32 / (tr32 / 1e3), 1), "tet_steps": int(steps32),
                     "roofline_frac_algorithmic": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic_bytes_per_launch": traffic,
                     **traffic_fractions(traffic, steps32 * BYTES_PER_TET_STEP, tr32)},
           "spp1024": {"ms": round(st1024["ms"], 3), "msamples_per_s": round(px * 1024 / (st1024["ms"] / 1e3) / 1e6, 3),
                       "tet_steps": int(st1024["tet_steps"])}}
    return out, (g, sc, ref)


def nrc_leg(tv, torch, grid, sc, frames: int, lr: float, ref=None, ref_spp: int = 1024,
            frames_per_row: int = 3, ema: float = 0.95) -> dict:
    """Online-trained radiance cache vs the plain renderer at equal RMSE.

    RMSE is measured against a 1024-spp plain render; that reference's own
    noise (the plain 32-spp noise scaled by 32/1024) is subtracted from every
    mean squared error.  The plain renderer's RMSE at any spp follows from
    its 32-spp RMSE by 1/sqrt(spp) and its time by spp (no fixed cost, which
    favours it): that model fills each row's side columns.  The headline
    figure is measured: the plain renderer at the spp whose measured RMSE is
    no worse than the 32-spp cache render's, timed.  A cache render's time
    includes its frame's training: the training paths ride the render
    launch, the Adam steps follow it."""
    import numpy as np
    cam, med, light = sc["camera"], sc["medium"], sc["light"]
    ro = sc["render"]
    if ref is None:
        ref, _ = tv.render(grid, cam, med, light, ref_spp, 7777, ro)
    ref = ref.cpu().numpy().astype(np.float64)
    a, sa = tv.render(grid, cam, med, light, 32, 1, ro)
    a = a.cpu().numpy().astype(np.float64)
    b, sb = tv.render(grid, cam, med, light, 32, 2, ro)
    b = b.cpu().numpy().astype(np.float64)
    var32 = float(((a - b) ** 2).mean()) / 2.0  # per-pixel variance of a 32-spp render
    mse_ref = var32 * 32.0 / ref_spp

    def rmse(img):
        return float(np.sqrt(max(float(((img - ref) ** 2).mean()) - mse_ref, 0.0)))

    rmse_plain32 = 0.5 * (rmse(a) + rmse(b))
    ms_plain32 = 0.5 * (sa["ms"] + sb["ms"])
    nrc = tv.Nrc(dict(lr=lr, ema=ema))
    p0 = nrc.export()
    untrained = None
    losses, train_ms = [], []
    for f in range(frames):
        st = nrc.train_frame(grid, cam, med, light, 50000 + f, ro)
        if f == 0:  # sigma_ref is set by the first frame; measure the untrained weights with it
            p1 = nrc.export()
            nrc.load(p0)
            img, _ = tv.render(grid, cam, med, light, 32, 3, dict(ro, nrc=nrc))
            untrained = rmse(img.cpu().numpy().astype(np.float64))
            nrc.load(p1)
        losses.append(st["loss"])
        train_ms.append(st["ms"])
    rows = []
    for i, spp in enumerate([1, 2, 4, 8, 16, 32, 128]):
        # frames of online rendering: the truncated render also traces the
        # frame's training paths in the same launch, then the cache trains;
        # RMSE and time averaged over `frames_per_row` consecutive frames
        mse, t, sts = 0.0, 0.0, []
        for f in range(frames_per_row):
            img, st = tv.render(grid, cam, med, light, spp, 4000 + 16 * i + f, dict(ro, nrc=nrc, nrc_train=1))
            e = rmse(img.cpu().numpy().astype(np.float64))
            mse += e * e / frames_per_row
            t += st["ms"] / frames_per_row
            sts.append(st)
        e = float(np.sqrt(mse))
        st = sts[-1]
        plain_spp = 32.0 * (rmse_plain32 / e) ** 2 if e > 0 else float("inf")
        plain_ms = ms_plain32 * plain_spp / 32.0
        rows.append({"spp": spp, "rmse": round(e, 6), "ms_frame": round(t, 3), "ms_trace": round(st["trace_ms"], 3),
                     "tet_steps": st["tet_steps"], "queries": st["cache_queries"],
                     "query_ms": round(st["cache_ms"], 3), "train_records": st["cache_records"],
                     "plain_spp_equal_rmse": round(plain_spp, 2), "plain_ms_equal_rmse": round(plain_ms, 3),
                     "speedup": round(plain_ms / t, 3)})
    best = max(rows[:-1], key=lambda r: r["speedup"])
    q = rows[5]
    # the headline row (32 spp with the cache) against the plain renderer
    # measured, not modelled: the plain render at the spp the model gives,
    # raised until its RMSE is no worse than the cache's
    plain_spp = int(np.ceil(q["plain_spp_equal_rmse"]))
    for _ in range(4):
        mse, t = 0.0, 0.0
        for f in range(frames_per_row):
            img, st = tv.render(grid, cam, med, light, plain_spp, 6000 + 16 * plain_spp + f, ro)
            e = rmse(img.cpu().numpy().astype(np.float64))
            mse += e * e / frames_per_row
            t += st["ms"] / frames_per_row
        e_plain = float(np.sqrt(mse))
        if e_plain <= q["rmse"] or plain_spp >= 4096:
            break
        plain_spp = int(np.ceil(plain_spp * (e_plain / q["rmse"]) ** 2 * 1.02))
    measured = {"cache_spp": q["spp"], "cache_rmse": q["rmse"], "cache_ms_frame": q["ms_frame"],
                "plain_spp": plain_spp, "plain_rmse": round(e_plain, 6), "plain_ms": round(t, 3),
                "speedup": round(t / q["ms_frame"], 3)}
    flops = q["queries"] * NRC_FLOP_PER_QUERY
    achieved = flops / (q["query_ms"] / 1e3) / 1e12 if q["query_ms"] > 0 else 0.0
    return {"speedup_equal_rmse": measured["speedup"], "at_spp": q["spp"], "measured": measured,
            "speedup_model_best": best["speedup"], "speedup_model_best_at_spp": best["spp"],
            "plain": {"spp": 32, "rmse": round(rmse_plain32, 6), "ms": round(ms_plain32, 3),
                      "tet_steps": sa["tet_steps"]},
            "reference_spp": ref_spp, "truncate_bounce": nrc.info()["truncate_bounce"],
            "train_frames": frames, "lr": lr, "weight_average": nrc.info()["ema"], "frames_per_row": frames_per_row,
            "train_frame_ms": round(float(np.mean(train_ms)), 3),
            "loss_first_last": [round(float(np.mean(losses[:5])), 5), round(float(np.mean(losses[-5:])), 5)],
            "rmse_untrained_32spp": round(untrained, 6), "bias_floor_rmse_128spp": rows[-1]["rmse"],
            "rows": rows,
            "query_roofline": {"bound": "mfma", "kernel": "k_nrc_query<1> (32 spp frame)",
                               "achieved": round(achieved, 3), "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                               "frac": round(achieved / MFMA_BF16_PEAK_TFLOPS, 5),
                               "flop_per_query": NRC_FLOP_PER_QUERY}}


def batch_leg(tv, torch, count: int, frames: int = 3) -> dict:
    """`count` scenes of the batch generator: one graph frame (all scenes'
    samples in one persistent launch), the same batch eagerly, and one
    tet_render call per scene in sequence; wall-clock per frame."""
    import numpy as np
    import synthetic
    sb = synthetic.scene_batch(count)
    grids, tets = [], 0
    for s in sb:
        g = tv.leb_build(torch.from_numpy(s["density_fn"]()).cuda(), s["n"], s["camera"], build=s["build"])
        tets += g.num_tets
        grids.append(g)
    cams = [s["camera"] for s in sb]
    media = [s["medium"] for s in sb]
    lights = [s["light"] for s in sb]
    spp = [s["render"]["spp"] for s in sb]
    ro = dict(max_bounces=sb[0]["render"]["max_bounces"])
    samples = sum(c["width"] * c["height"] * k for c, k in zip(cams, spp))
    b = tv.Batch(grids, cams, media, lights, spp, ro)

    def timed(fn):
        fn(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = None
        for f in range(frames):
            out = fn(1 + f)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / frames, out

    ms_graph, st = timed(lambda f: b.render([s["seed"] + 1000 * f for s in sb]))
    ms_eager, _ = timed(lambda f: tv.render_batch(grids, cams, media, lights, spp,
                                                  [s["seed"] + 1000 * f for s in sb], ro, outs=b.outs))

    def sequential(f):
        for i, s in enumerate(sb):
            tv.render(grids[i], cams[i], media[i], lights[i], spp[i], s["seed"] + 1000 * f, ro, out=b.outs[i])
    ms_seq, _ = timed(sequential)
    return {"scenes": count, "samples_per_frame": int(samples), "tets_total": int(tets),
            "ms_graph_frame": round(ms_graph, 3), "ms_eager_batch": round(ms_eager, 3),
            "ms_sequential_calls": round(ms_seq, 3), "speedup_graph_vs_sequential": round(ms_seq / ms_graph, 3),
            "msamples_per_s_graph": round(samples / (ms_graph / 1e3) / 1e6, 3),
            "tet_steps_per_frame": int(st["tet_steps"]),
            "tet_steps_per_s_graph": round(st["tet_steps"] / (ms_graph / 1e3), 1)}


def calibrate_copy(torch):
    """A plain device copy of COPY_BYTES: the counters' scale reference."""
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--render-only", action="store_true", help="time only the render (grid built once)")
    ap.add_argument("--calibrate-copy", action="store_true", help="end with a plain 1 GiB device copy")
    ap.add_argument("--no-nrc", action="store_true", help="skip the radiance-cache leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-scene batch leg")
    ap.add_argument("--no-autotune", action="store_true", help="use the fixed launch options")
    ap.add_argument("--launch", default=None,
                    help="JSON launch options for the tracing kernel (skips the autotuner), e.g. the ones a "
                         "previous run chose")
    ap.add_argument("--no-dda", action="store_true", help="skip the regular-grid (DDA) leg")
    ap.add_argument("--regular-grid-1024", action="store_true",
                    help="also render the cloud resampled to 1024^3 with both renderers (the paper's "
                         "comparison at its resolution)")
    ap.add_argument("--no-channels", action="store_true", help="skip the extra-channel leg")
    ap.add_argument("--no-camera-path", action="store_true", help="skip the moving-camera (leb_update) leg")
    ap.add_argument("--no-density-models", action="store_true", help="skip the density-model leg")
    ap.add_argument("--no-plume", action="store_true",
                    help="skip the 1024^3 plume leg (the radiance-cache leg then runs on the cloud)")
    ap.add_argument("--nrc-frames", type=int, default=100)
    ap.add_argument("--nrc-lr", type=float, default=1e-2)
    ap.add_argument("--nrc-ema", type=float, default=0.99)
    ap.add_argument("--plume-only", action="store_true",
                    help="run only the 1024^3 plume leg (its build and 32 / 1024 spp renders) and print its figures")
    ap.add_argument("--host-rounds", action="store_true",
                    help="build with every round driven from the host (no cooperative launch; the grid is the "
                         "same): for runs under rocprofv3, which fails at exit after a cooperative launch")
    ap.add_argument("--summarize-pmc", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "OUT"))
    ap.add_argument("--summarize-trace", nargs=2, metavar=("TRACE_DIR", "OUT"))
    ap.add_argument("--summarize-counters", nargs=2, metavar=("PMC_DIR", "OUT"))
    ap.add_argument("--steps-per-launch", type=float, default=0.0)
    ap.add_argument("--command", default="")
    ap.add_argument("--workload", default="", help="workload named in a counter summary")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc, args.command, *( [args.workload] if args.workload else []))
        return
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace, args.command)
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, args.command, args.steps_per_launch)
        return
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (got --gpus {args.gpus}): the method's hot path is "
              "single-GPU here; sharding across GPUs (sample ranges per GPU, one image reduce) is not built.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synthetic
    import paper_2506_11510_amd as tv

    if args.plume_only:
        plume, _ = plume_leg(tv, torch, args.host_rounds, json.loads(args.launch) if args.launch else None)
        if args.calibrate_copy:
            calibrate_copy(torch)
        print(json.dumps({"plume": plume}), flush=True)
        return

    sc = synthetic.scene("cloud")
    if args.host_rounds:
        sc["build"] = dict(sc["build"], host_rounds=1)
    # launch configuration of the tracing kernel: the library's autotuner
    # times probe renders of this frame (8 spp) from this starting point
    # (the library's defaults: one sample per work item, batches of 64
    # items per wave, 256-thread blocks, compact 32-byte records, 5 waves
    # per SIMD, events once 32 lanes wait)
    sc["render"] = dict(sc["render"], samples_per_item=1, batch_items=64, block_size=256, record_layout=32,
                        waves_per_simd=5, event_wait=32)
    cam, spp = sc["camera"], sc["render"]["spp"]
    d = sc["density_fn"]()
    dev = torch.from_numpy(d).cuda()
    out = torch.empty((cam["height"], cam["width"], 3), dtype=torch.float32, device="cuda")
    tune_ms = None
    if args.launch:
        sc["render"] = dict(sc["render"], **json.loads(args.launch))
    elif not args.no_autotune:
        g0 = tv.leb_build(dev, sc["n"], cam, build=sc["build"])
        # probes render the timed frame itself (its spp): shorter probes
        # favour launch shapes that are slower on the full frame
        sc["render"], tune_ms = tv.autotune(g0, cam, sc["medium"], sc["light"], sc["render"], probe_spp=spp)
        del g0
    torch.cuda.synchronize()

    def step(seed):
        g = tv.leb_build(dev, sc["n"], cam, build=sc["build"])
        _, st = tv.render(g, cam, sc["medium"], sc["light"], spp, seed, sc["render"], out=out)
        return g, st

    grid = None
    if args.render_only:
        grid = tv.leb_build(dev, sc["n"], cam, build=sc["build"])
    for i in range(args.warmup):
        if args.render_only:
            tv.render(grid, cam, sc["medium"], sc["light"], spp, 100 + i, sc["render"], out=out)
        else:
            step(100 + i)
    torch.cuda.synchronize()
    build_ms, render_ms, trace_ms, tet_steps, infos = [], [], [], [], []
    t0 = time.perf_counter()
    for i in range(args.steps):
        if args.render_only:
            _, st = tv.render(grid, cam, sc["medium"], sc["light"], spp, 1000 + i, sc["render"], out=out)
            info = grid.info()
        else:
            g, st = step(1000 + i)
            info = g.info()
        build_ms.append(info["ms"])
        render_ms.append(st["ms"])
        trace_ms.append(st["trace_ms"])
        tet_steps.append(st["tet_steps"])
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    samples = cam["width"] * cam["height"] * spp
    value = samples / (ms_per_step / 1e3) / 1e6
    mean_render_ms = float(np.mean(render_ms))
    mean_trace_ms = float(np.mean(trace_ms))
    mean_steps = float(np.mean(tet_steps))
    # roofline of the dominant kernel: algorithmic bytes of one launch over
    # its HIP-event duration on the launch stream
    achieved = mean_steps * BYTES_PER_TET_STEP / (mean_trace_ms / 1e3) / 1e9
    img = out.cpu().numpy()
    res = {
        "metric": METRIC, "value": round(value, 3), "unit": "Msamples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "256^3 fBm cloud (seed 1, 20% occupancy, sigma_t max 20) -> adaptive LEB grid "
                               "(1 px target, tau 0.2, depth <= 24) -> 1024x1024, 32 spp, 32 bounces, albedo 0.9, "
                               "HG g 0.3, sun + env, analytic light transmittance",
                   "step": "render only" if args.render_only else "leb_build + tet_render",
                   "num_tets": infos[-1]["num_tets"], "max_depth": infos[-1]["max_depth"],
                   "build_rounds": infos[-1]["rounds"], "parallelism": "1 GPU",
                   "launch": {k: sc["render"][k] for k in tv.TUNED_FIELDS}, "autotune_probe_ms": tune_ms},
        "tet_steps_per_s": round(mean_steps / (mean_render_ms / 1e3), 1),
        "tet_steps_per_s_trace_kernel": round(mean_steps / (mean_trace_ms / 1e3), 1),
        "render_ms": round(mean_render_ms, 3), "trace_kernel_ms": round(mean_trace_ms, 3),
        "build_ms": round(float(np.mean(build_ms)), 3),
        "render_only_msamples_per_s": round(samples / (mean_render_ms / 1e3) / 1e6, 3),
        "tet_steps_per_frame": int(mean_steps),
        "events_per_frame": {k: int(st[k]) for k in ("real_collisions", "null_collisions", "escapes", "truncated",
                                                      "light_rays_queued")},
        "image_mean": float(img.mean()),
        "roofline": {"bound": "hbm",
                     "kernel": "k_render<TetMedium%s, %d, 0, false, false> + queued light rays (k_light, sort)"
                               % ("32" if sc["render"]["record_layout"] == 32 else "", sc["render"]["waves_per_simd"]),
                     "achieved": round(achieved, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(sc["render"]),
                     "algorithmic_bytes_per_launch": int(mean_steps * BYTES_PER_TET_STEP),
                     **traffic_fractions(measured_traffic(sc["render"]), mean_steps * BYTES_PER_TET_STEP,
                                         mean_trace_ms),
                     "note": "the cloud grid's compact records (32 B x %d tets = %.0f MB) fit the 256 MB "
                             "Infinity Cache, so this is a cache-resident figure; the plume leg's (records "
                             "streaming from HBM) is plume.spp32.roofline_frac_algorithmic"
                             % (infos[-1]["num_tets"], infos[-1]["num_tets"] * 32 / 1e6)},
        "cpu_baseline": None,
    }
    if not args.no_dda:
        res["dda"] = dda_leg(tv, dev, sc)
        res["dda"]["tet_vs_dda_render_speedup"] = round(res["dda"]["ms"] / mean_render_ms, 3)
    res["host_buffers"] = host_io_leg(tv, torch, d, sc)
    if args.regular_grid_1024:
        res["regular_grid_1024"] = regular_grid_1024_leg(tv, torch, dev, sc)
    if not args.no_camera_path:
        res["camera_path"] = camera_path_leg(tv, torch, dev, sc)
    if not args.no_batch:
        res["batch"] = batch_leg(tv, torch, 64)
    if grid is None:
        grid = tv.leb_build(dev, sc["n"], cam, build=sc["build"])
    if not args.no_channels:
        res["channels"] = channels_leg(tv, torch, grid, sc, mean_render_ms)
    if not args.no_density_models:
        res["density_models"] = density_model_leg(tv, torch, dev, sc, mean_render_ms)
    del dev
    plume = None
    if not args.no_plume:
        res["plume"], plume = plume_leg(tv, torch, args.host_rounds)
    if not args.no_nrc:
        if plume is not None:  # the cache study runs on the production-scale scene
            del grid
            g, psc, ref = plume
            res["nrc"] = nrc_leg(tv, torch, g, psc, args.nrc_frames, args.nrc_lr, ref=ref, ref_spp=1024,
                                 ema=args.nrc_ema)
            res["nrc"]["scene"] = "plume 1024^3 (64 bounces)"
        else:
            res["nrc"] = nrc_leg(tv, torch, grid, sc, args.nrc_frames, args.nrc_lr, ema=args.nrc_ema)
            res["nrc"]["scene"] = "cloud 256^3 (32 bounces)"
    if args.calibrate_copy:
        calibrate_copy(torch)
    if not args.no_cpu_baseline:
        # the host threads this process may use: one GPU's share of the
        # host's cores (16 per GPU), whatever os.cpu_count() reports
        n_threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        res["cpu_baseline"] = cpu_baseline(sc, d, n_threads)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
