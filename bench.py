"""Benchmark: spacetime simplices tested per second for critical-point tracking on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload noise1024] [--no-cpu-baseline]

One step = one ftk_track_cp2d/3d call over the whole series (detection of every n-simplex, compaction,
sublocation, classification, union-find stitching, labels) with the input already resident in HBM.  Prints one
JSON line.  The roofline entry describes the kernel with the largest share of the step, timed with HIP events that
the library records on the call's stream (ftk_options.profile).
"""
import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4  # wave64 VALU instructions/s

WORKLOADS = {
    "blobs64": "2D scalar 64x64x10, 8 moving Gaussians, seed 0",
    "noise1024": "2D scalar 1024x1024x100, 256 moving Gaussians + N(0,1e-3) noise, seed 1",
    "levels1024": "2D scalar 1024x1024x100, the noisy blob field rounded to 16 levels",
    "blobs3d256": "3D scalar 256x256x256x16, 512 moving Gaussians, seed 2",
    "vortex4096": "2D vector 4096x4096x50, 1024 moving sources/sinks/vortices, seed 4",
    "batch96": "96 uneven 2D scalar series (nx, ny log-uniform 128-2048, 8-64 steps), seeds 3+i; batched vs plain",
    "iso_blobs3d256": "isovolume f = 0.5 of the 3D scalar 256x256x256x16 blob series (512 moving Gaussians, seed 2)",
    "vortex_waves512": "vortex surfaces of a 3D complex 512x128x64x8 series (independent random cosine waves for the "
                       "real and imaginary parts, 8 each, seed 6)",
    "mesh500k": "2D vector field on a 500,000-point Delaunay mesh of [0,100]^2 extruded over 40 steps (moving "
                "sources and vortices, seed 9)",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="noise1024", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-post", action="store_true", help="skip the trajectory post-processing timings")
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload only: skip the other configurations' precision and batch reports")
    ap.add_argument("--cpu-steps", type=int, default=0, help="time steps of the oracle sample (0: automatic)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (counter calibration) and exit")
    return ap.parse_args()


def calibrate_copy(mib):
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_bytes": n * 4, "launches": 3}), flush=True)


def source_hash(names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2011_08697_amd", "csrc", n), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


KERNEL_SOURCES = {
    "detect2d": ["cp2d.hip", "common.h", "kuhn.h"], "emit2d": ["cp2d.hip", "common.h", "kuhn.h"],
    "uf_label": ["uf.hip", "common.h"], "scan": ["scan.hip"],
    "detect3d": ["cp3d.hip", "common.h", "kuhn.h"], "emit3d": ["cp3d.hip", "common.h", "kuhn.h"],
}


def measured_counters(kernel, workload):
    """Counter summary of the kernel from the committed rocprofv3 runs (HBM bytes and VALU instructions per launch),
    if it was taken on the current source; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            d = json.load(fh)
        if d.get("source_hash") != source_hash(KERNEL_SOURCES[kernel]):
            return None
        return d
    except Exception:
        return None


def batch_compare(F, synth, dev, steps, warmup):
    """The 96-series workload: one batched call (one persistent launch per stage for all series) against 96 plain
    calls, each timed over `steps` repetitions after `warmup`.  Returns (report, fields, tested simplices)."""
    import torch
    t0 = time.time()
    fields = synth.batch_series(count=96, seed0=3, device=dev)
    gen_s = time.time() - t0
    ts = [torch.from_numpy(f).to(dev) for f in fields]
    steps_total = sum(f.shape[0] for f in fields)
    tested = sum(F.simplex_count(2, (f.shape[2], f.shape[1], f.shape[0])) for f in fields)

    # tilings tuned per series shape first (untimed); plain calls use their own, the batched launch its largest's
    for t in ts:
        F.autotune_cp2d(t)
    torch.cuda.synchronize()

    def batched():
        res = F.track_cp2d_batched(ts)
        return sum(r["n_hits"] for r in res)

    def plain():
        return sum(F.track_cp2d(t)["n_hits"] for t in ts)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            nh = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps, nh

    tb, nhb = timed(batched)
    tp, nhp = timed(plain)
    assert nhb == nhp
    # kernel phases of one batched call (HIP events on the stream)
    st = F.track_cp2d_batched(ts, profile=1)[0]["stats"]
    torch.cuda.synchronize()
    phases = {"detect2d": round(st["t_detect_ms"], 3), "scan": round(st["t_scan_ms"], 3),
              "emit2d": round(st["t_emit_ms"], 3), "uf_link": round(st["t_link_ms"], 3)}
    steps_total = sum(f.shape[0] for f in fields)
    rep = {"workload": WORKLOADS["batch96"], "series": len(fields), "time_steps_total": steps_total,
           "vertices_total": int(sum(f.size for f in fields)), "n_hits": nhb, "generation_s": round(gen_s, 1),
           "batched": {"steps_per_s": round(steps_total / tb, 1), "ms_per_batch": round(tb * 1e3, 3),
                       "phase_ms": phases},
           "plain": {"steps_per_s": round(steps_total / tp, 1), "ms_per_batch": round(tp * 1e3, 3)},
           "batched_over_plain": round(tp / tb, 3), "timed_calls": steps}
    return rep, tested, tb


def bench_batched(args, F, synth, dev):
    """Batched form (one persistent launch per stage for all 96 series) against 96 plain calls."""
    rep, tested, tb = batch_compare(F, synth, dev, args.steps, args.warmup)
    line = {
        "metric": "spacetime simplices tested/s + HBM roofline frac; batched vs plain steps/s",
        "value": round(tested / tb, 1), "unit": "simplices/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(tb * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {k: rep[k] for k in ("workload", "series", "time_steps_total", "vertices_total", "n_hits",
                                       "generation_s")},
        "batched": rep["batched"], "plain": rep["plain"], "batched_over_plain": rep["batched_over_plain"],
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def precision_report(F, field_np, field, kind, n, sample=20000):
    """Per-result error of the default FP32 path (FP32 sublocation and classification, FP64 only where the FP32
    type is not certified) against binary64: over every hit against the library's FP64 mode (precision = 1, the
    oracle's binary64 operation order), and over a sample of hits against the oracle itself."""
    import numpy as np
    import torch
    from oracle import oracle as O
    run = (lambda **kw: F.track_cp2d(field, kind=kind, **kw)) if n == 2 else (lambda **kw: F.track_cp3d(field, **kw))
    r = run()
    r64 = run(precision=1)
    torch.cuda.synchronize()
    same_faces = r["n_hits"] == r64["n_hits"] and bool(torch.equal(r["face_id"], r64["face_id"]))
    p32, p64 = r["pos"].double(), r64["pos"].double()
    rel = (p32 - p64).abs() / p64.abs().clamp(min=1.0)
    nh = r["n_hits"]
    all_hits = {"hits": nh, "faces_identical": same_faces,
                "type_agree": float((r["type"] == r64["type"]).double().mean()) if nh else 1.0,
                "labels_identical": bool(torch.equal(r["label"], r64["label"])),
                "pos_rel_err_max": float(rel.max()) if nh else 0.0,
                "pos_rel_err_mean": float(rel.mean()) if nh else 0.0}
    fid = r["face_id"].cpu().numpy()
    pos = r["pos"].cpu().numpy().astype(np.float64)
    typ = r["type"].cpu().numpy()
    flg = r["flags"].cpu().numpy()
    rng = np.random.default_rng(0)
    idx = rng.choice(len(fid), min(sample, len(fid)), replace=False)
    ev = O.eval_faces(field_np, fid[idx], n=n, kind=kind)
    err = np.abs(pos[idx] - ev["pos"]) / np.maximum(1.0, np.abs(ev["pos"]))
    oracle = {"sampled": int(len(idx)), "punctured_agree": bool(np.all(ev["punctured"] == 1)),
              "type_agree": float(np.mean(typ[idx] == ev["type"])), "pos_rel_err_max": float(err.max()),
              "pos_rel_err_mean": float(err.mean())}
    return {"vs_fp64_mode_all_hits": all_hits, "vs_oracle_sample": oracle, "tolerance": 1e-5,
            "fp64_fallback_frac": float(np.mean((flg & 2) != 0)) if nh else 0.0,
            "degenerate_frac": float(np.mean((flg & 1) != 0)) if nh else 0.0}


def bench_iso(args, F, synth, dev):
    """Isovolume tracking (edge pass, pentachoron unions, tessellation, labels) of the 3D blob series: K calls of
    ftk_track_iso3d on the resident field; value = spacetime edges tested per second."""
    import numpy as np
    import torch
    field = torch.from_numpy(synth.make("blobs3d256", device=dev)).to(dev)
    nt, nz, ny, nx = field.shape
    dims = (nx, ny, nz, nt)
    c = 0.5
    L = F.lib()
    stream = torch.cuda.current_stream(dev)
    sh = ctypes.c_void_p(stream.cuda_stream)
    pool = F._TorchPool(dev)
    opt = F._options(pool)

    def one():
        r = F.IsoResult()
        st = L.ftk_track_iso3d(ctypes.c_void_p(field.data_ptr()), nx, ny, nz, nt, c, ctypes.byref(opt), sh,
                               ctypes.byref(r))
        if st != 0:
            raise F.FtkError(st, F.last_error())
        out = (int(r.n_hits), int(r.n_components), int(r.n_tets))
        L.ftk_iso_result_free(ctypes.byref(r), ctypes.byref(opt), sh)
        return out

    for _ in range(args.warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        nh, ncomp, ntets = one()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = el * 1e3 / args.steps
    edges = F.edge_count(dims)
    V = int(np.prod(dims))
    alg = 4 * V + 32 * nh + 16 * ntets  # field in; edge id, position and label per crossing; 4 int32 per tet
    line = {
        "metric": "spacetime edges tested/s (isovolume tracking)", "value": round(edges / (ms * 1e-3), 1),
        "unit": "edges/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOADS["iso_blobs3d256"], "dims": list(dims), "isovalue": c, "n_hits": nh,
                   "n_components": ncomp, "n_tets": ntets, "edges_per_step": edges},
        "roofline": {"bound": "hbm", "kernel": "whole call", "achieved": round(alg / (ms * 1e-3) / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        from oracle import iso as OI
        sample = np.ascontiguousarray(field[:2, :24, :24, :24].cpu().numpy())
        t0 = time.perf_counter()
        OI.track_iso(sample, c)
        cpu_s = time.perf_counter() - t0
        se = F.edge_count((24, 24, 24, 2))
        line["cpu_baseline"] = {"value": round(se / cpu_s, 1), "unit": "edges/s", "cores": 1, "kind": "oracle",
                                "sample": f"24x24x24x2 corner of the same series ({se} edges, numpy, {cpu_s:.1f} s)"}
    print(json.dumps(line), flush=True)


def bench_vortex(args, F, synth, dev):
    """Vortex surface tracking of a random-wave complex series at the grid shape of the paper's superconductivity
    case: K calls of ftk_track_vortex3d on the resident series; value = spacetime triangles tested per second."""
    import numpy as np
    import torch
    psi_np = synth.random_waves_3d(512, 128, 64, 8, seed=6)
    psi = torch.from_numpy(psi_np).to(dev)
    nt, _, nz, ny, nx = psi.shape
    dims = (nx, ny, nz, nt)
    L = F.lib()
    sh = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    pool = F._TorchPool(dev)
    opt = F._options(pool)

    def one():
        r = F.VortexResult()
        st = L.ftk_track_vortex3d(ctypes.c_void_p(psi.data_ptr()), nx, ny, nz, nt, ctypes.byref(opt), sh,
                                  ctypes.byref(r))
        if st != 0:
            raise F.FtkError(st, F.last_error())
        out = (int(r.n_hits), int(r.n_components))
        L.ftk_vortex_result_free(ctypes.byref(r), ctypes.byref(opt), sh)
        return out

    for _ in range(args.warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        nh, ncomp = one()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    tris = F.triangle_count(dims)
    V = int(np.prod(dims))
    alg = 8 * V + 32 * nh  # complex field in (two binary32 per vertex); id 8 B, point 16 B, label 8 B per positive
    line = {
        "metric": "spacetime triangles tested/s (vortex surface tracking)", "value": round(tris / (ms * 1e-3), 1),
        "unit": "triangles/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": WORKLOADS["vortex_waves512"], "dims": list(dims), "n_hits": nh,
                   "n_components": ncomp, "triangles_per_step": tris},
        "roofline": {"bound": "hbm", "kernel": "whole call", "achieved": round(alg / (ms * 1e-3) / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        from oracle import vortex as OV
        sample = np.ascontiguousarray(psi_np[:2, :, :6, :10, :12])
        t0 = time.perf_counter()
        OV.track_vortex(sample)
        cpu_s = time.perf_counter() - t0
        st_ = F.triangle_count((12, 10, 6, 2))
        line["cpu_baseline"] = {"value": round(st_ / cpu_s, 1), "unit": "triangles/s", "cores": 1, "kind": "oracle",
                                "sample": f"12x10x6x2 corner of the same series ({st_} triangles, python, {cpu_s:.1f} s)"}
    print(json.dumps(line), flush=True)


def bench_mesh(args, F, synth, dev):
    """Critical points on an extruded unstructured mesh: K calls of ftk_track_cp_mesh on a mesh handle (topology
    built once) and a resident field; value = spacetime faces tested per second (S per step, interval faces for all
    but the last step)."""
    import numpy as np
    import torch
    xy, tri = synth.delaunay_mesh(500000, extent=100.0, seed=9)
    nt = 40
    rng = np.random.Generator(np.random.PCG64(9))
    P = xy.astype(np.float64) / 10.0
    f = np.zeros((nt, 2, len(xy)), np.float64)
    for _ in range(16):
        c, v, rot = rng.uniform(1, 9, 2), rng.uniform(-0.1, 0.1, 2), rng.uniform(0, np.pi)
        for t in range(nt):
            d = P - (c + v * t)
            w = np.exp(-(d ** 2).sum(1) / 2.0)
            f[t, 0] += w * (np.cos(rot) * d[:, 0] - np.sin(rot) * d[:, 1])
            f[t, 1] += w * (np.sin(rot) * d[:, 0] + np.cos(rot) * d[:, 1])
    dxy = torch.from_numpy(xy).to(dev)
    dtri = torch.from_numpy(np.ascontiguousarray(tri, np.int32)).to(dev)
    dfield = torch.from_numpy(f.astype(np.float32)).to(dev)
    L = F.lib()
    sh = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    pool = F._TorchPool(dev)
    opt = F._options(pool)

    mesh = ctypes.c_void_p()  # topology built once, outside the timed calls (as a mesh is set up once per dataset)
    st0 = L.ftk_mesh_create(ctypes.c_void_p(dxy.data_ptr()), len(xy), ctypes.c_void_p(dtri.data_ptr()), len(tri), sh,
                            ctypes.byref(mesh))
    if st0 != 0:
        raise F.FtkError(st0, F.last_error())

    def one():
        r = F.MeshResult()
        st = L.ftk_track_cp_mesh(mesh, ctypes.c_void_p(dfield.data_ptr()), nt, ctypes.byref(opt), sh,
                                 ctypes.byref(r))
        if st != 0:
            raise F.FtkError(st, F.last_error())
        out = (int(r.n_hits), int(r.n_trajectories), int(r.faces_per_step), int(r.n_edges))
        L.ftk_mesh_result_free(ctypes.byref(r), ctypes.byref(opt), sh)
        return out

    for _ in range(args.warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        nh, ntraj, S, ne = one()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    L.ftk_mesh_destroy(mesh)
    nf = len(tri)
    faces = nt * nf + (nt - 1) * (2 * ne + 2 * nf)
    alg = 8 * len(xy) * nt + 12 * nf + 8 * len(xy) + 28 * nh  # field, mesh in; id, point, label out
    line = {
        "metric": "spacetime faces tested/s (critical points on an extruded triangle mesh)",
        "value": round(faces / (ms * 1e-3), 1), "unit": "faces/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": WORKLOADS["mesh500k"], "vertices": len(xy), "triangles": nf, "edges": ne, "steps": nt,
                   "n_hits": nh, "n_trajectories": ntraj, "faces_per_call": faces},
        "roofline": {"bound": "hbm", "kernel": "whole call", "achieved": round(alg / (ms * 1e-3) / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        from oracle import mesh as OM
        sub = np.nonzero((xy[:, 0] < 12.0) & (xy[:, 1] < 12.0))[0]  # a corner patch of the same mesh and field
        keep = np.all(np.isin(tri, sub), axis=1)
        remap = -np.ones(len(xy), np.int64)
        remap[sub] = np.arange(len(sub))
        stri = remap[tri[keep]]
        sf = np.ascontiguousarray(f[:3][:, :, sub].astype(np.float32))
        t0 = time.perf_counter()
        OM.track_cp_mesh(xy[sub], stri, sf)
        cpu_s = time.perf_counter() - t0
        se = len(OM.mesh_edges(stri))
        sfaces = 3 * len(stri) + 2 * (2 * se + 2 * len(stri))
        line["cpu_baseline"] = {"value": round(sfaces / cpu_s, 1), "unit": "faces/s", "cores": 1, "kind": "oracle",
                                "sample": f"{len(sub)}-vertex corner patch of the same mesh, 3 steps ({sfaces} faces, "
                                          f"python, {cpu_s:.1f} s)"}
    print(json.dumps(line), flush=True)


def post_report(F, field, n, kind, dims, reps=2):
    """Wall time of each trajectory post-processing call on this workload's result (after the timed region; not part
    of value): table, slice at the middle step, loop filter, order, smoothing (half window 2), simplification."""
    import torch
    res = F.track_cp2d(field, kind=kind) if n == 2 else F.track_cp3d(field)
    torch.cuda.synchronize()
    ms = {}
    for _ in range(reps):  # the first pass also grows torch's cache; keep the last
        def timed(name, fn):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            ms[name] = round((time.perf_counter() - t0) * 1e3, 3)
            return out
        tab = timed("table", lambda: F.trajectory_table(res, dims))
        timed("slice", lambda: F.slice_at(res, dims, dims[-1] // 2))
        timed("filter_loops", lambda: F.filter_loops(res, tab, 1.0))
        order, off = timed("order", lambda: F.trajectory_order(res, dims, tab))
        sm = timed("smooth", lambda: F.smooth_types(res, tab, order, off, 2))
        si = timed("simplify", lambda: F.simplify_types(res, tab, order, off, 1.0))
    nh = res["n_hits"]
    lengths = (off[1:] - off[:-1]) if tab["n"] else off[:0]
    return {"ms": ms, "n_hits": nh, "n_trajectories": tab["n"],
            "longest": int(lengths.max()) if tab["n"] else 0,
            "order_hits_per_s": round(nh / (ms["order"] * 1e-3), 1) if ms["order"] > 0 else None,
            "smoothed": int((sm != res["type"]).sum()), "simplified": int((si != res["type"]).sum())}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (a series would shard by time "
              "slabs); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return

    import numpy as np
    import torch

    import paper_2011_08697_amd as F
    from paper_2011_08697_amd import synth

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    wl = args.workload
    if wl == "batch96":
        return bench_batched(args, F, synth, dev)
    if wl == "iso_blobs3d256":
        return bench_iso(args, F, synth, dev)
    if wl == "vortex_waves512":
        return bench_vortex(args, F, synth, dev)
    if wl == "mesh500k":
        return bench_mesh(args, F, synth, dev)
    n = 3 if wl == "blobs3d256" else 2
    kind = 1 if wl == "vortex4096" else 0
    t0 = time.time()
    field_np = synth.make(wl, device=dev if wl in ("blobs3d256", "vortex4096") else None)
    gen_s = time.time() - t0
    field = torch.from_numpy(field_np).to(dev)
    if n == 2:
        dims = (field_np.shape[-1], field_np.shape[-2], field_np.shape[0])
    else:
        dims = (field_np.shape[3], field_np.shape[2], field_np.shape[1], field_np.shape[0])
    L = F.lib()
    stream = torch.cuda.current_stream(dev)
    sh = ctypes.c_void_p(stream.cuda_stream)
    # outputs come from torch's caching allocator through the library's allocator hooks (as for any torch user)
    pool = F._TorchPool(dev)
    opt = F._options(pool, profile=1)

    def one_step():
        r = F.Result()
        if n == 2:
            st = L.ftk_track_cp2d(ctypes.c_void_p(field.data_ptr()), kind, dims[0], dims[1], dims[2],
                                  ctypes.byref(opt), sh, ctypes.byref(r))
        else:
            st = L.ftk_track_cp3d(ctypes.c_void_p(field.data_ptr()), 0, dims[0], dims[1], dims[2], dims[3],
                                  ctypes.byref(opt), sh, ctypes.byref(r))
        if st != 0:
            raise F.FtkError(st, F.last_error())
        out = (int(r.n_hits), int(r.n_trajectories), int(r.stats.simplices_tested),
               r.stats.t_detect_ms, r.stats.t_scan_ms, r.stats.t_emit_ms, r.stats.t_link_ms,
               int(r.stats.fp64_fallbacks), int(r.stats.degenerate_sublocations))
        L.ftk_result_free(ctypes.byref(r), ctypes.byref(opt), sh)  # returns the output tensors to torch's cache
        return out

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    phase = np.zeros(4)
    t_start = time.perf_counter()
    for _ in range(args.steps):
        nh, ntraj, tested, td, ts, te, tl, n_fp64, n_degen = one_step()
        phase += (td, ts, te, tl)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed * 1e3 / args.steps
    value = tested * args.steps / elapsed
    phase /= args.steps

    # dominant kernel and its algorithmic bytes per launch
    V = int(np.prod(dims))
    in_bytes = V * 4 * (n if kind == 1 else 1)
    rec = 22 if n == 2 else 26  # face_id 8 + pos 4*(n+1) + type 1 + flags 1
    names = ["detect%dd" % n, "scan", "emit%dd" % n, "uf_label"]  # uf_label: hooking + labels (8 B per hit out)
    alg = [in_bytes, 0, rec * nh, 8 * nh]
    k = int(np.argmax(phase))
    kernel = names[k]
    achieved = alg[k] / (phase[k] * 1e-3) / 1e9 if phase[k] > 0 else 0.0
    counters = measured_counters(kernel, wl)
    traffic = float(counters["bytes_per_launch"]) if counters else None
    # VALU busy: wave64 VALU instructions per launch over the issue capacity in the measured duration
    # (256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles per wave64 instruction)
    valu_busy = None
    if counters and counters.get("valu_insts_per_launch") and phase[k] > 0:
        valu_busy = round(counters["valu_insts_per_launch"] / (phase[k] * 1e-3 * VALU_ISSUE_PEAK), 3)
    roofline = {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "valu_busy": valu_busy,
                "traffic_source": (f"profiles/traffic_{kernel}_{wl}.json: rocprofv3 FETCH_SIZE / WRITE_SIZE and SQ "
                                   f"counters of the committed source (not measured in this run)") if counters else
                                  "none: the committed counter runs predate this source",
                "avg_ms": round(float(phase[k]), 4),
                "phase_ms": {nm: round(float(p), 4) for nm, p in zip(names, phase)},
                "path_frac": round((in_bytes + (rec + 8) * nh) / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    cpu = None
    if not args.no_cpu_baseline and n == 2:
        from oracle import oracle as O
        cores = min(16, len(os.sched_getaffinity(0)))
        steps = args.cpu_steps or (20 if wl in ("noise1024", "levels1024") else 3)
        if wl == "blobs64":
            sample = field_np
        else:
            sample = np.ascontiguousarray(field_np[:steps])
        t0 = time.perf_counter()
        tr = O.track(sample, n=2, kind=kind, nthreads=cores)
        cpu_s = time.perf_counter() - t0
        cpu = {"value": round(tr.simplices_tested / cpu_s, 1), "unit": "simplices/s", "cores": cores,
               "kind": "oracle",
               "sample": f"first {sample.shape[0]} of {field_np.shape[0]} time steps of the same field "
                         f"({tr.simplices_tested} simplices, {tr.n_hits} hits, full detect + sublocate + stitch, "
                         f"{cpu_s:.1f} s)"}

    post = None if args.no_post else post_report(F, field, n, kind, dims)

    precision = None
    if wl in ("vortex4096", "blobs3d256", "noise1024"):
        precision = {wl: precision_report(F, field_np, field, kind, n)}
    batch = None
    if wl == "noise1024" and not args.no_extras:
        # the other configurations' evidence on the default run: FP32-vs-FP64 errors of the 4096^2 vector series
        # and the 256^3 3D series, and the 96-series batched-over-plain ratio (outside the timed region)
        del field
        torch.cuda.empty_cache()
        for other in ("vortex4096", "blobs3d256"):
            o_np = synth.make(other, device=dev)
            o_dev = torch.from_numpy(o_np).to(dev)
            precision[other] = precision_report(F, o_np, o_dev, 1 if other == "vortex4096" else 0,
                                                3 if other == "blobs3d256" else 2,
                                                sample=20000 if other == "vortex4096" else 2000)
            del o_np, o_dev
            torch.cuda.empty_cache()
        batch, _, _ = batch_compare(F, synth, dev, steps=5, warmup=2)

    line = {
        "metric": "spacetime simplices tested/s + HBM roofline frac; batched vs plain steps/s",
        "value": round(value, 1), "unit": "simplices/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": WORKLOADS[wl], "dims": list(dims), "kind": "vector" if kind else "scalar",
                   "n_hits": nh, "n_trajectories": ntraj, "simplices_per_step": tested,
                   "fp64_fallbacks": n_fp64, "degenerate_sublocations": n_degen,
                   "generation_s": round(gen_s, 1)},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if post is not None:
        line["post"] = post
    if precision is not None:
        line["precision"] = precision
    if batch is not None:
        line["batch96"] = batch
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
