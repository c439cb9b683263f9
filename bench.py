"""Throughput of the smooth-part single-layer potential on one MI355X.

One step = one pass of the whole hot path on the resident workload: charges
q = w g (set_density), gridding, the pruned 3-D FFT with the fused kernel
multiplier, the inverse FFT and the interpolation at the nodes
(eval_single_layer). Metric: (M_q + N) points per second, M_q quadrature
sources and N nodes, stated with the relative L2 error against the FP64
oracle's definition of the smooth part (the NDFT route: no window, no FFT).

Default line: the thin film 1 x 1 x 0.02 at spacing 1/512 (1,089,536
triangles, 3,268,608 sources, 544,770 nodes, seeded smooth magnetisation, seed
3) on the anisotropic 1024 x 1024 x 64 grid, in FP64 at the window and cut-off
that slp_choose_cutoff picks for a relative error of 1e-6, with its error
measured on the 10,000 stored oracle nodes (tests/golden/film512_phi_sample.npz).
Extra keys of the same line: the film with the Gaussian window at the same
gate and in FP32, the 64-cell cube, 64 densities on the cube in one launch, a
batch of 32 icospheres, the served Poisson mix (p50/p99) beside the plain FP64
path, and the oracle timed on the host. Usage:
  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload film512|cube64|sphere_l3]
                  [--precision fp64|fp32] [--window gauss|kb] [--m M] [--tol T]
                  [--near-tol T] [--no-extras] [--serve] [--mix32] [--potential]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {  # published MI355X figures
    "hbm_GBps": 8000.0,
    "f64_vector_TFLOPs": 78.6,
    "f64_matrix_TFLOPs": 78.6,
    "f32_vector_TFLOPs": 157.3,
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--m", type=int, default=None)
    ap.add_argument("--tol", type=float, default=None,
                    help="pick window and m with slp_choose_cutoff for this relative error")
    ap.add_argument("--window", choices=["gauss", "kb"], default=None,
                    help="Gaussian or Kaiser-Bessel; by default (and for a missing --m) "
                         "slp_choose_cutoff picks them for --tol")
    ap.add_argument("--workload", default="film512")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the main line (no film/cube/batched/served/oracle extras)")
    ap.add_argument("--volume-targets", action="store_true",
                    help="cube64 only: evaluate at all (65^3) nodes of the structured "
                         "tetrahedral mesh of the cube instead of the boundary nodes")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle", action="store_true")
    ap.add_argument("--graph", action="store_true",
                    help="replay the evaluation through a captured HIP graph")
    ap.add_argument("--batch", type=int, default=1,
                    help="densities per step on the one geometry (batched launch)")
    ap.add_argument("--serve", action="store_true",
                    help="served mix: Poisson request stream through the request server")
    ap.add_argument("--mix32", action="store_true",
                    help="multi-mesh batch: 32 icospheres of levels 2-6 in one batched call")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--discard", type=int, default=100,
                    help="served mix: first requests left out of the latency figures")
    ap.add_argument("--integrated", type=int, default=0,
                    help="grid the window integrated over each triangle (the paper's matrix A, "
                         "Sec. 3.1) with this many Gauss points per direction; 0 = point sources")
    ap.add_argument("--near-storage", choices=["context", "fp64", "fp32"], default="context",
                    help="precision the near-field values are stored in (the context's by "
                         "default; fp32 in an FP64 context halves the bytes of the HBM-bound "
                         "product, the sums stay FP64)")
    ap.add_argument("--near-tol", type=float, default=None,
                    help="add the near-field correction with eps from slp_near_radius(tol)")
    ap.add_argument("--potential", action="store_true",
                    help="Alg. 1 computation phase on the tetrahedral mesh of the 64-cell cube: "
                         "phi_1 (P1 FEM, conjugate gradients), d phi_1/dn, the density, phi_2 "
                         "at all 274,625 nodes with the near field (--near-tol, default 1e-3), "
                         "phi = phi_1 + phi_2")
    ap.add_argument("--cg-tol", type=float, default=1e-8,
                    help="relative residual of the phi_1 solve (--potential)")
    ap.add_argument("--precond", choices=["jacobi", "amg"], default="amg",
                    help="preconditioner of the phi_1 solve (--potential): diagonal, or a "
                         "smoothed-aggregation multigrid V-cycle")
    ap.add_argument("--rotate-deg", type=float, default=0.0,
                    help="--potential as a time stepper: the magnetisation turns by this angle "
                         "(degrees, about the axis (1,1,1)) every step and phi_1 starts from the "
                         "previous step's solution")
    ap.add_argument("--rho", type=float, default=0.8, help="offered load / capacity")
    ap.add_argument("--autotune", default=None, metavar="CACHE",
                    help="time the gridding split candidates before the timed region and use "
                         "the fastest (cube workloads and --mix32); results are cached in this "
                         "JSON file ('-' for no file)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="first copy this many MiB device-to-device (a kernel of known "
                         "traffic, to scale hardware byte counters)")
    return ap.parse_args()


def algorithmic_units(stage, info, m, esz):
    """(amount, unit, bound) of algorithmic work of one launch of `stage`.

    spread_bins: 2 (2m)^3 + (2m)^2 flops per source (tensor-product accumulate);
    spread_reduce: the grid region written once (the per-bin blocks it sums are
    an artefact of the method, not algorithmic traffic);
    interp: 2 (2m)^3 + (2m)^2 flops per node; FFT passes: bytes read + written
    by the pass over the pruned region (complex = 2 esz bytes)."""
    w = 2 * m
    R = info["extent"]
    n = info["_n"]
    Kx, Ky, Kz = n[0] // 2 + 1, n[1] + 1, n[2] + 1
    c = 2 * esz
    if stage == "spread_bins" and info.get("_iw_stored"):
        # integrated-window gridding: the stored window integrals read once
        # (value and column), the row offsets, the density read and its
        # element means written and read once, the region grid written
        st = info["_iw_stored"]
        colb = 2 * st + 4 * (st // 256) if info["_iw_packed"] else 4 * st
        rows = R[0] * R[1] * R[2]
        M = info["n_src"] // 3
        return (st * esz + colb + (rows + 1) * 8 + rows * esz + info["n_src"] * 8 + 2 * M * 8,
                "byte", "hbm")
    if stage == "spread_bins":
        # FP64 with 2m = 16 accumulates each run on the matrix cores
        bound = "mfma" if esz == 8 and w == 16 else "alu"
        return info["n_src"] * (2.0 * w ** 3 + w ** 2), "flop", bound
    if stage == "spread_reduce":
        return R[0] * R[1] * R[2] * esz, "byte", "hbm"
    if stage == "interp":
        return info["n_targets"] * (2.0 * w ** 3 + w ** 2), "flop", "alu"
    if stage == "fft_x_fwd":
        return R[2] * R[1] * (R[0] * esz + Kx * c), "byte", "hbm"
    if stage == "fft_y_fwd":
        return R[2] * Kx * (R[1] * c + Ky * c), "byte", "hbm"
    if stage == "fft_z_mul_inv":
        return Kx * Ky * (2 * R[2] * c + Kz * esz), "byte", "hbm"
    if stage == "fft_y_inv":
        return R[2] * Kx * (Ky * c + R[1] * c), "byte", "hbm"
    if stage == "fft_x_inv":
        return R[2] * R[1] * (Kx * c + R[0] * esz), "byte", "hbm"
    if stage == "near":
        # the stored matrix read once (per entry the value and a 16-bit packed
        # or 32-bit column, per 256-entry chunk a 32-bit base when packed), the
        # row offsets, the density (3 M values) read once, phi read and written
        nt = info["n_targets"]
        st = info["_stored"]
        colb = 2 * st + 4 * (st // 256) if info["_packed"] else 4 * st
        vsz = info.get("_near_esz", esz)
        return (st * vsz + colb + (nt + 1) * 8 + info["n_src"] * 8 + 16 * nt, "byte", "hbm")
    raise KeyError(stage)


def code_only(src):
    """C++ source without comments and with whitespace collapsed: what the
    compiler sees, so that a comment edit does not invalidate measurements."""
    import re
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def measured_traffic(key, stage, nb):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE runs (profiles/traffic.json: counters scaled by what
    they read for a device copy of known size), looked up by workload key, or
    None when no run covers this configuration or the kernel sources (without
    comments) have changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if nb != 1 or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    for src, sha in rec["sources_sha256"].items():
        with open(os.path.join(ROOT, src)) as f:
            if hashlib.sha256(code_only(f.read()).encode()).hexdigest() != sha:
                return None
    e = rec["entries"].get(key)
    if e is None or e.get("stage") != stage:
        return None
    return e["bytes_per_launch"]


def traffic_key(workload, precision, window, m, near_tol=None, near_storage=None,
                integrated=0):
    key = f"{workload}/{precision}/{window}/m{m}"
    if near_tol is not None:
        key += f"/near{near_tol:g}"
        if near_storage not in (None, "context", precision):
            key += f"/stored{near_storage}"
    if integrated:
        key += f"/integrated{integrated}"
    return key


def host_cpu():
    """Host facts for the CPU baselines: logical CPUs, the CPUs this process may
    use, and the CPU model."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": usable, "logical_cpus": os.cpu_count(), "model": model}


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        return os.cpu_count()


def served_mix(args, rhos, requests, discard):
    """Served mix (config: Poisson stream over resident geometries, icosphere
    L3-L6 and cubes of 16-256 cells per edge, a fresh seeded magnetisation per
    request from a pool of densities per shape): FP32 through the request
    server at offered loads rho x capacity, p50/p99 latency and pts/s, the
    first `discard` requests of each run left out; beside it the plain FP64
    path (one stream, one solve after the other) on the same mix. Window and
    cut-off: slp_choose_cutoff at 1e-4 (FP32) and 1e-6 (FP64)."""
    import torch

    import paper_1305_3162_amd as slp
    from synth import icosphere, cube, RandomSmoothMagnetisation, density_from_magnetisation
    from synth.workloads import expsum_interval

    w32, m32 = slp.choose_cutoff(1e-4, slp.FP32)
    w64, m64 = slp.choose_cutoff(1e-6, slp.FP64)
    shapes = [("sphere", L) for L in (3, 4, 5, 6)] + [("cube", c) for c in (16, 32, 64, 128, 256)]
    rng = np.random.default_rng(5)
    geo = []
    for kind, size in shapes:
        nodes, tris = icosphere(size) if kind == "sphere" else cube(size)
        N = grid_rule(nodes, tris)
        r_lo, r_hi = expsum_interval(nodes)
        w, g = slp.expsum_sinc(0.2, r_lo, r_hi, 1e-12)
        dens = []
        for k in range(2):
            mf = RandomSmoothMagnetisation(5000 + 10 * len(geo) + k, nodes.min(0), nodes.max(0))
            dens.append(torch.as_tensor(density_from_magnetisation(nodes, tris, mf), device="cuda"))
        geo.append(dict(kind=kind, size=size, nodes=nodes, tris=tris, N=N, w=w, g=g, dens=dens,
                        pts=3 * tris.shape[0] + nodes.shape[0]))
    budget = 8 << 30
    srv = slp.Server(budget, 4)
    for G in geo:
        G["id"] = srv.add_geometry(G["nodes"], G["tris"], (G["N"],) * 3, m32, G["w"], G["g"], 2,
                                   slp.FP32, window=w32)
        G["phi"] = [torch.empty(G["nodes"].shape[0], dtype=torch.float64, device="cuda")
                    for _ in range(8)]
    torch.cuda.synchronize()
    t_setup = time.perf_counter()
    for G in geo:            # build every geometry once (setup is not part of a request)
        srv.wait(srv.submit(G["id"], G["dens"][0], G["phi"][0]), 120)
    t_setup = time.perf_counter() - t_setup
    # capacity at saturation: 200 requests submitted at once
    picks0 = rng.integers(len(geo), size=200)
    srv.stats(reset=True)
    t0 = time.perf_counter()
    tks = [srv.submit(geo[i]["id"], geo[i]["dens"][0], geo[i]["phi"][k % 8])
           for k, i in enumerate(picks0)]
    for tk in tks:
        srv.wait(tk, 120)
    cap = 200 / (time.perf_counter() - t0)
    runs = []
    picks_all = []
    for rho in rhos:
        picks = rng.integers(len(geo), size=requests)
        picks_all.append(picks)
        lam = rho * cap
        arrive = np.cumsum(rng.exponential(1.0 / lam, size=requests))
        srv.stats(reset=True)
        tks = []
        reset_done = discard <= 0
        t0 = time.perf_counter()
        for k, i in enumerate(picks):
            while time.perf_counter() - t0 < arrive[k]:
                if not reset_done and k > discard and srv.poll(tks[discard - 1]):
                    srv.stats(reset=True)
                    reset_done = True
            G = geo[i]
            tks.append(srv.submit(G["id"], G["dens"][k % 2], G["phi"][k % 8]))
        if not reset_done:
            srv.wait(tks[discard - 1], 120)
            srv.stats(reset=True)
        for tk in tks:
            srv.wait(tk, 120)
        st = srv.stats()
        runs.append({"rho": rho, "offered_rate_per_s": round(lam, 1),
                     "p50_ms": round(st["p50_s"] * 1e3, 4), "p99_ms": round(st["p99_s"] * 1e3, 4),
                     "mean_ms": round(st["mean_s"] * 1e3, 4),
                     "pts_per_s": round(st["pts_per_s"], 1), "completed_counted": st["completed"],
                     "failed": st["failed"], "setups": st["setups"],
                     "evictions": st["evictions"]})
    srv.close()
    # plain FP64 path on the same mix, one stream
    plain = []
    for G in geo:
        gg = slp.Geometry(G["nodes"], G["tris"], (G["N"],) * 3, m64, G["w"], G["g"], 2, slp.FP64,
                          window=w64)
        phi = torch.empty(G["nodes"].shape[0], dtype=torch.float64, device="cuda")
        for _ in range(3):
            gg.set_density(G["dens"][0])
            gg.eval(phi)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(10):
            gg.set_density(G["dens"][0])
            gg.eval(phi)
        torch.cuda.synchronize()
        plain.append((time.perf_counter() - t1) / 10)
        gg.close()
    picks = np.concatenate(picks_all)
    mix_pts = float(np.mean([geo[i]["pts"] for i in picks]))
    mix_time64 = float(np.mean([plain[i] for i in picks]))
    wname = {slp.WINDOW_GAUSS: "gauss", slp.WINDOW_KB: "kb"}
    return {
        "metric": "served SL-potential NUFFT latency and (M+N) pts/s",
        "dtype": "f32", "window": wname[w32], "m": m32, "runs": runs,
        "capacity_per_s": round(cap, 1), "requests_per_run": requests,
        "discarded_per_run": discard, "setup_all_geometries_s": round(t_setup, 2),
        "plain_fp64": {"pts_per_s": round(mix_pts / mix_time64, 1), "window": wname[w64],
                       "m": m64, "mean_ms_per_request": round(mix_time64 * 1e3, 4)},
        "config": {"workload": "Poisson stream over icosphere L3-L6 and cubes 16/32/64/128/256 "
                               "cells per edge (uniform pick, seed 5), 2 seeded magnetisations "
                               "per shape, grid clamp(prevpow2(1/mean scaled edge), 64, 512)^3",
                   "slots": 4, "budget_bytes": budget},
    }


def serve(args):
    rec = served_mix(args, [args.rho], args.requests, args.discard)
    rec["n_gpus"] = 1
    rec["higher_is_better"] = True
    rec["data"] = "synthetic"
    print(json.dumps(rec), flush=True)


def grid_rule(nodes, tris):
    """N_q = clamp(prevpow2(1 / mean scaled edge), 64, 512) (scaled into (-0.2, 0.2))."""
    e = nodes[tris[:, [1, 2, 0]]] - nodes[tris]
    hbar = 0.4 * float(np.linalg.norm(e, axis=2).mean()) / float((nodes.max(0) - nodes.min(0)).max())
    return int(min(512, max(64, 2 ** int(np.floor(np.log2(1.0 / hbar))))))


def multi_mesh(args, prec, window, m, steps, warmup):
    """Multi-mesh batch: 32 icospheres, levels uniform in {2..6} (seed 4100), each with
    its own seeded magnetisation (seeds 4101-4132) and grid by the rule above, evaluated
    by one slp_eval_batched_mode call per step with fused launches (one launch per stage
    for all meshes); beside it the same batch with the per-mesh launch sequences
    overlapped on the library's four streams, and the items one after the other on one
    stream."""
    import torch

    import paper_1305_3162_amd as slp
    from synth import icosphere, RandomSmoothMagnetisation, density_from_magnetisation
    from synth.workloads import expsum_interval

    levels = np.random.default_rng(4100).integers(2, 7, size=32)
    geos, dens, phis, pts = [], [], [], 0
    cache = {}
    for i, L in enumerate(levels):
        if L not in cache:
            nodes, tris = icosphere(int(L))
            r_lo, r_hi = expsum_interval(nodes)
            w, g = slp.expsum_sinc(0.2, r_lo, r_hi, 1e-12)
            cache[L] = (nodes, tris, w, g, grid_rule(nodes, tris))
        nodes, tris, w, g, N = cache[L]
        share, cells = 0, 0
        if args.autotune:
            t = tuned_share(args, nodes, tris, (N,) * 3, m, w, g, 2, prec, 37.0, window, None)
            share, cells = t["seg_share"], t["reduce_cells"]
        geos.append(slp.Geometry(nodes, tris, (N,) * 3, m, w, g, 2, prec, window=window,
                                 seg_share=share, reduce_cells=cells))
        mf = RandomSmoothMagnetisation(4101 + i, nodes.min(0), nodes.max(0))
        dens.append(torch.as_tensor(density_from_magnetisation(nodes, tris, mf), device="cuda"))
        phis.append(torch.empty(nodes.shape[0], dtype=torch.float64, device="cuda"))
        pts += 3 * tris.shape[0] + nodes.shape[0]
    handles = [G.handle for G in geos]
    stream = torch.cuda.current_stream()

    def batched():
        slp.eval_batched(handles, dens, phis, stream, mode=slp.BATCH_FUSED)

    def lanes():
        slp.eval_batched(handles, dens, phis, stream, mode=slp.BATCH_LANES)

    def one_by_one():
        for G, d, p in zip(geos, dens, phis):
            G.set_density(d, stream)
            G.eval(p, stream)

    out = {}
    for name, fn in (("batched", batched), ("lanes", lanes), ("one_by_one", one_by_one)):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        out[name] = (time.perf_counter() - t0) / steps
    for G in geos:
        G.close()
    return {
        "metric": "multi-mesh batched SL-potential NUFFT (M+N) pts/s",
        "value": round(pts / out["batched"], 1), "unit": "pts/s",
        "steps": steps, "warmup": warmup, "ms_per_step": round(out["batched"] * 1e3, 5),
        "dtype": "f64" if prec == slp.FP64 else "f32",
        "window": "kb" if window == slp.WINDOW_KB else "gauss", "m": m,
        "launches": "fused: one launch per stage for all meshes (FFT passes per line length)",
        "lanes_pts_per_s": round(pts / out["lanes"], 1),
        "lanes_ms_per_step": round(out["lanes"] * 1e3, 5),
        "one_by_one_pts_per_s": round(pts / out["one_by_one"], 1),
        "one_by_one_ms_per_step": round(out["one_by_one"] * 1e3, 5),
        "config": {"workload": "32 icospheres, levels uniform in 2..6 (seed 4100), seeded "
                               "magnetisations 4101-4132, grid clamp(prevpow2(1/mean scaled "
                               "edge), 64, 512)^3 per mesh",
                   "levels": [int(x) for x in levels], "points": pts,
                   "gridding_split": "autotuned" if args.autotune else "automatic"},
    }


def mix32(args):
    import torch

    import paper_1305_3162_amd as slp
    torch.cuda.init()          # the device is set up by torch before the library allocates
    torch.cuda.synchronize()
    prec = slp.FP64 if args.precision == "fp64" else slp.FP32
    window, m = resolve_window(args, slp, prec)
    rec = multi_mesh(args, prec, window, m, args.steps, args.warmup)
    rec.update({"n_gpus": 1, "higher_is_better": True, "data": "synthetic"})
    print(json.dumps(rec), flush=True)


def potential(args):
    """One step = Alg. 1's computation phase (slp_scalar_potential): phi_1 by
    preconditioned conjugate gradients from zero, d phi_1/dn, the element density, phi_2 at
    every node of the tetrahedral mesh (smooth part + near field), the sum."""
    import torch

    import paper_1305_3162_amd as slp
    from synth import cube_tets, RandomSmoothMagnetisation
    from synth.workloads import expsum_interval

    prec = slp.FP64 if args.precision == "fp64" else slp.FP32
    m_win = args.m if args.m is not None else (8 if prec == slp.FP64 else 5)
    near_tol = 1e-3 if args.near_tol is None else args.near_tol
    nodes, tets = cube_tets(64)
    mf = RandomSmoothMagnetisation(2, nodes.min(0), nodes.max(0))
    m_nodes = mf(nodes)
    lo, hi = expsum_interval(nodes)
    w, g = slp.expsum_sinc(0.2, lo, hi, 1e-12)
    stream = torch.cuda.current_stream()
    t1 = time.perf_counter()
    F = slp.Fem(nodes, tets, stream)
    t_fem_setup = time.perf_counter() - t1
    t1 = time.perf_counter()
    slp.fem_set_preconditioner(F.handle, args.precond, stream)
    t_precond_setup = time.perf_counter() - t1
    G = slp.Geometry(nodes, F.boundary, (128, 128, 128), m_win, w, g, 2, prec)
    t1 = time.perf_counter()
    eps = G.near_radius(near_tol) if near_tol > 0 else 0.0
    storage = near_storage(args, slp, prec)
    if eps > 0:
        G.setup_near_field(eps, stream, storage)
    t_near_setup = time.perf_counter() - t1
    nf = G.near_field_info()
    phi = torch.empty(nodes.shape[0], dtype=torch.float64, device="cuda")
    warm = args.rotate_deg != 0.0
    n_in = args.warmup + args.steps if warm else 1
    # every step's magnetisation resident in HBM before the timed region: the
    # field turned by k * rotate_deg about (1,1,1) (Rodrigues' rotation)
    ax = np.ones(3) / np.sqrt(3.0)
    mds = []
    for k in range(n_in):
        th = np.deg2rad(args.rotate_deg * k)
        mk = (m_nodes * np.cos(th) + np.cross(ax, m_nodes) * np.sin(th)
              + np.outer(m_nodes @ ax, ax) * (1.0 - np.cos(th)))
        mds.append(torch.as_tensor(mk, device="cuda"))
    iters_all = []
    for k in range(args.warmup):
        iters_all.append(slp.scalar_potential(F.handle, G.handle, mds[k if warm else 0], phi,
                                              args.cg_tol, 20000, warm and k > 0, stream))
    torch.cuda.synchronize()
    slp.set_timing(G.handle, 1)
    slp.stage_times(G.handle, reset=True)
    iters_all = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        kk = args.warmup + k
        iters_all.append(slp.scalar_potential(F.handle, G.handle, mds[kk if warm else 0], phi,
                                              args.cg_tol, 20000, warm and kk > 0, stream))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    iters = int(round(float(np.mean(iters_all))))
    md = mds[args.warmup + args.steps - 1 if warm else 0]
    m_nodes = md.cpu().numpy()
    stage_ms, cnt = slp.stage_times(G.handle, reset=True)
    slp.set_timing(G.handle, False)
    ms_per_step = wall * 1e3 / args.steps
    avg = {k: v / max(cnt, 1) for k, v in stage_ms.items()}
    phi2_ms = sum(avg.values())
    n_src = 3 * F.boundary.shape[0]
    pts = n_src + nodes.shape[0]
    info = dict(G.info)
    info["_n"] = [64, 64, 64]
    info["_stored"], info["_packed"] = nf["stored"], nf["packed"]
    info["_near_esz"] = 8 if storage == slp.FP64 else 4
    esz = 8 if prec == slp.FP64 else 4
    dom = max(avg, key=avg.get)
    amount, unit, bound = algorithmic_units(dom, info, m_win, esz)
    dur_s = max(avg[dom] * 1e-3, 1e-12)
    if bound == "hbm":
        achieved, peak, runit = amount / dur_s / 1e9, PEAK["hbm_GBps"], "GB/s"
    else:
        achieved = amount / dur_s / 1e12
        peak = PEAK["f64_vector_TFLOPs"] if prec == slp.FP64 else PEAK["f32_vector_TFLOPs"]
        if bound == "mfma":
            peak = PEAK["f64_matrix_TFLOPs"]
        runit = "TFLOP/s"
    roofline = {"bound": bound, "achieved": round(achieved, 4), "peak": peak, "unit": runit,
                "frac": round(achieved / peak, 5), "traffic": None, "kernel": dom,
                "avg_launch_us": round(avg[dom] * 1e3, 3)}
    out = phi.cpu().numpy()
    rel_err, cpu_baseline = None, None
    if not args.no_oracle:
        from oracle import direct, fem, geometry, nearfield as nfo
        t1 = time.perf_counter()
        phi1 = fem.solve_phi1(nodes, tets, m_nodes, "cg")
        tris, owner = fem.boundary_faces(nodes, tets)
        dn = fem.dphi1_dn(nodes, tets, phi1, tris, owner)
        dens = geometry.density_p1(nodes, tris, m_nodes, dn)
        prob = direct.prepare(nodes, tris, dens, (128, 128, 128), 2, 0.2, lo, hi, 1e-12, 37.0)
        far = direct.phi_ndft(prob)
        t_bulk = time.perf_counter() - t1
        rows = np.random.default_rng(7).choice(nodes.shape[0], 8, replace=False)
        t1 = time.perf_counter()
        near = np.zeros(rows.size)
        if eps > 0:
            rp_o, cols_o, _ = nfo.near_pairs(nodes, tris, nodes[rows], eps)
            vals_o = nfo.near_values(prob, nodes, tris, nodes[rows], rp_o, cols_o)
            gbar = nfo.element_mean_density(prob, tris.shape[0])
            nz = np.diff(rp_o) > 0
            near[nz] = np.add.reduceat(vals_o * gbar[cols_o], rp_o[:-1][nz]) / nfo.FOUR_PI
        t_row = (time.perf_counter() - t1) / rows.size
        ref = phi1[rows] + far[rows] + near
        rel_err = float(np.abs(out[rows] - ref).max() / np.abs(phi1 + far).max())
        if not args.no_cpu_baseline:
            t_solve = t_bulk + t_row * nodes.shape[0]
            cpu_baseline = {"value": round(pts / t_solve, 2), "unit": "pts/s", "cores": os.cpu_count(),
                            "kind": "oracle",
                            "sample": f"oracle Alg. 1: phi_1 by preconditioned CG (scipy) on the whole "
                                      f"mesh, the NDFT route of phi_2 at all {nodes.shape[0]} nodes "
                                      f"({t_bulk:.1f} s together), and the near-field rows timed on 8 "
                                      f"rows ({t_row:.3f} s per row) scaled to all rows"}
    rec = {
        "metric": "complete scalar potential, Alg. 1 computation phase (M+N) pts/s",
        "value": round(pts / (ms_per_step * 1e-3), 1), "unit": "pts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == slp.FP64 else "f32", "data": "synthetic",
        "config": {"workload": f"tetrahedral mesh of the unit cube, 64 cells per edge: "
                               f"{nodes.shape[0]} nodes, {tets.shape[0]} tetrahedra, "
                               f"{F.info['n_free']} free nodes, {F.boundary.shape[0]} boundary "
                               f"triangles ({n_src} sources), seeded smooth magnetisation (seed 2), "
                               f"grid 128^3, Gaussian m={m_win}",
                   "cg_tol": args.cg_tol, "cg_iterations": iters, "precond": args.precond,
                   "precond_setup_s": round(t_precond_setup, 3),
                   "time_stepping": ({"rotate_deg_per_step": args.rotate_deg,
                                      "warm_start": True} if warm else None),
                   "near_field": {"tol": near_tol, "eps": round(eps, 6), "pairs": nf["nnz"],
                                  "stored": nf["stored"], "setup_s": round(t_near_setup, 2),
                                  "values_stored_as": "fp64" if storage == slp.FP64 else "fp32"},
                   "fem_setup_s": round(t_fem_setup, 2), "points": pts},
        "phi2_ms": round(phi2_ms, 4), "phi1_and_rest_ms": round(ms_per_step - phi2_ms, 4),
        "stage_us": {k: round(v * 1e3, 3) for k, v in avg.items()},
        "rel_err_vs_oracle": rel_err,
        "err_kind": "max |error| over 8 seeded nodes / max |phi| (oracle phi_1 by CG to 1e-13)",
        "roofline": roofline, "cpu_baseline": cpu_baseline,
    }
    print(json.dumps(rec), flush=True)
    G.close()
    F.close()


def near_storage(args, slp, prec):
    """Storage precision of the near-field values for --near-storage."""
    return {"context": prec, "fp64": slp.FP64, "fp32": slp.FP32}[args.near_storage]


def tuned_share(args, nodes, tris, grid, m, w, g, alpha, prec, eta2, window, targets):
    """The autotuner's split and block-sum form for this workload (timed now or
    read from the cache)."""
    from paper_1305_3162_amd import autotune
    cache = None if args.autotune == "-" else args.autotune
    r = autotune.tune_share(nodes, tris, grid, m, w, g, alpha, prec, eta2, window=window,
                            targets=targets, cache=cache)
    return {"seg_share": r["seg_share"], "reduce_cells": r["reduce_cells"],
            "auto_share": r["auto_share"], "auto_cells": r["auto_cells"], "cached": r["cached"],
            "candidates_us": {f'{c["seg_share"]}/{c["reduce_cells"]}': round(c["us"], 2)
                              for c in r["candidates"]}}


GATE = {"fp64": 1e-6, "fp32": 1e-4}   # stated relative L2 tolerances
GOLDEN = os.path.join(ROOT, "tests", "golden", "film512_phi_sample.npz")


def resolve_window(args, slp, prec):
    """(window, m): as given, or what slp_choose_cutoff picks for --tol (default:
    the precision's gate), over both windows unless --window names one."""
    win = {"gauss": slp.WINDOW_GAUSS, "kb": slp.WINDOW_KB}
    if args.m is not None:
        return win[args.window or "gauss"], args.m
    tol = args.tol if args.tol is not None else GATE[args.precision]
    return slp.choose_cutoff(tol, prec, None if args.window is None else win[args.window])


def timed_steps(torch, slp, geom, step, steps, warmup, stream, every=16):
    """Warm-up, then `steps` steps bracketed by device synchronisation; every
    `every`-th step records per-stage HIP events on the evaluation stream.
    Returns (ms per step, average per-stage ms, number of recorded steps)."""
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    slp.set_timing(geom.handle, every)
    slp.stage_times(geom.handle, reset=True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage_ms, cnt = slp.stage_times(geom.handle, reset=True)
    slp.set_timing(geom.handle, False)
    ms = max(wall * 1e3, ev0.elapsed_time(ev1)) / steps
    avg = {k: v / max(cnt, 1) for k, v in stage_ms.items()}
    return ms, avg, cnt


def golden_error(wl, geom, phi):
    """Relative L2 error of phi on the stored oracle nodes of the film (the
    oracle's definition route, written by tests/golden/make_film512_golden.py),
    after checking that the stored instance is this one."""
    gold = np.load(GOLDEN)
    if int(gold["terms"]) != geom.info["terms_kept"] or not np.allclose(
            geom.info["scale"], gold["s"], rtol=1e-15):
        raise RuntimeError("stored oracle values belong to another instance")
    idx = gold["idx"]
    ref = gold["phi"]
    return float(np.linalg.norm(phi[idx] - ref) / np.linalg.norm(ref)), int(idx.size)


def roofline_of(stage, avg, info, m, esz, nb, prec_fp64, key, cnt):
    """Roofline record of the dominant stage from its event-timed average."""
    if cnt == 0:
        return None
    amount, unit, bound = algorithmic_units(stage, info, m, esz)
    amount *= nb
    dur_s = max(avg[stage] * 1e-3, 1e-12)
    if bound == "hbm":
        achieved, peak, runit = amount / dur_s / 1e9, PEAK["hbm_GBps"], "GB/s"
    else:
        achieved = amount / dur_s / 1e12
        peak = PEAK["f64_vector_TFLOPs"] if prec_fp64 else PEAK["f32_vector_TFLOPs"]
        if bound == "mfma":
            peak = PEAK["f64_matrix_TFLOPs"]
        runit = "TFLOP/s"
    traffic = measured_traffic(key, stage, nb)
    return {"bound": bound, "achieved": round(achieved, 4), "peak": peak, "unit": runit,
            "frac": round(achieved / peak, 5), "traffic": traffic,
            "traffic_source": "profiles/traffic.json (rocprofv3 FETCH_SIZE/WRITE_SIZE of this "
                              "kernel source, scaled by a device copy)" if traffic else None,
            "kernel": stage, "avg_launch_us": round(avg[stage] * 1e3, 3),
            "algorithmic": {"amount_per_launch": amount, "unit": unit}}


def workload_text(wl, n_tgt, window, m, targets):
    wname = "Kaiser-Bessel" if window == 1 else "Gaussian"
    if wl.name.startswith("film"):
        body = (f"thin film 1 x 1 x 0.02 at spacing 1/512, seeded smooth magnetisation "
                f"(seed 3)")
    elif wl.name.startswith("cube"):
        body = "unit cube 64x64 cells per face, seeded smooth magnetisation (seed 2)"
    else:
        body = wl.name
    return (f"{wl.name}: {body}, {wl.tris.shape[0]} triangles, {wl.n_nodes} nodes, "
            f"{wl.n_src} quadrature sources, "
            + (f"{n_tgt} targets (all nodes of the structured tetrahedral mesh), "
               if targets is not None else "")
            + f"grid {wl.grid[0]}x{wl.grid[1]}x{wl.grid[2]}, alpha 2, {wname} window "
              f"cut-off m={m}")


def solve_line(args, slp, torch, wl, prec, window, m, steps, warmup, err="auto"):
    """One workload at one precision/window/m: timed steps, stage times, the
    dominant kernel's roofline and the error against the oracle (film: stored
    nodes; others: the definition at every node)."""
    stream = torch.cuda.current_stream()
    w, g = slp.expsum_sinc(wl.es_h, wl.es_r_lo, wl.es_r_hi, wl.es_tol)
    t1 = time.perf_counter()
    geom = slp.Geometry(wl.nodes, wl.tris, wl.grid, m, w, g, wl.alpha, prec, wl.eta2,
                        window=window)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t1
    dens = torch.as_tensor(wl.dens, device="cuda")
    phi = torch.empty(geom.info["n_targets"], dtype=torch.float64, device="cuda")

    def step():
        geom.set_density(dens, stream)
        geom.eval(phi, stream)

    ms, avg, cnt = timed_steps(torch, slp, geom, step, steps, warmup, stream)
    out = phi.cpu().numpy()
    info = dict(geom.info)
    info["_n"] = [wl.grid[q] // wl.alpha for q in range(3)]
    esz = 8 if prec == slp.FP64 else 4
    pname = "fp64" if prec == slp.FP64 else "fp32"
    wname = "kb" if window == slp.WINDOW_KB else "gauss"
    dom = max(avg, key=avg.get) if cnt else "spread_bins"
    rec = {"value": round((wl.n_src + wl.n_nodes) / (ms * 1e-3), 1), "ms_per_step": round(ms, 5),
           "precision": pname, "window": wname, "m": m,
           "stage_us": {k: round(v * 1e3, 3) for k, v in avg.items()},
           "roofline": roofline_of(dom, avg, info, m, esz, 1, prec == slp.FP64,
                                   traffic_key(wl.name, pname, wname, m), cnt),
           "setup_s": round(t_setup, 3),
           "gridding_split": {"seg_share": int(info["seg_share"]),
                              "segments": int(info["n_segments"]),
                              "reduce_cells": int(info["reduce_cells"])}}
    if err == "golden":
        e, n = golden_error(wl, geom, out)
        rec["rel_l2_err_vs_oracle"] = e
        rec["err_kind"] = f"relative L2 over {n} stored oracle nodes (definition route)"
    elif err == "full":
        from oracle import direct
        ref = direct.phi_ndft(direct.prepare_workload(wl))
        rec["rel_l2_err_vs_oracle"] = float(np.linalg.norm(out - ref) / np.linalg.norm(ref))
        rec["err_kind"] = "relative L2 over all nodes (oracle definition route)"
    geom.close()
    return rec


def batched_densities(args, slp, torch, wl, prec, window, m, nb, steps, warmup):
    """nb seeded densities on one geometry per step, one slp_eval_batched call."""
    from synth import RandomSmoothMagnetisation, density_from_magnetisation
    stream = torch.cuda.current_stream()
    w, g = slp.expsum_sinc(wl.es_h, wl.es_r_lo, wl.es_r_hi, wl.es_tol)
    geom = slp.Geometry(wl.nodes, wl.tris, wl.grid, m, w, g, wl.alpha, prec, wl.eta2,
                        window=window)
    dl = [torch.as_tensor(density_from_magnetisation(
        wl.nodes, wl.tris, RandomSmoothMagnetisation(4000 + k, wl.nodes.min(0),
                                                     wl.nodes.max(0))), device="cuda")
          for k in range(nb)]
    pl = [torch.empty(wl.n_nodes, dtype=torch.float64, device="cuda") for _ in range(nb)]
    hl = [geom.handle] * nb

    def step():
        slp.eval_batched(hl, dl, pl, stream)

    ms, avg, cnt = timed_steps(torch, slp, geom, step, steps, warmup, stream)
    geom.close()
    return {"value": round(nb * (wl.n_src + wl.n_nodes) / (ms * 1e-3), 1),
            "ms_per_step": round(ms, 5), "densities": nb,
            "precision": "fp64" if prec == slp.FP64 else "fp32",
            "window": "kb" if window == slp.WINDOW_KB else "gauss", "m": m,
            "config": {"workload": f"{wl.name}, {nb} seeded magnetisations (seeds "
                                   f"4000-{4000 + nb - 1}) per step in one batched call"}}


def cpu_baseline_r3(wl, m, window_name, npts):
    """The oracle's plain CPU NUFFT (R3: the same gridding / FFT / deconvolution /
    NFFT steps with the same window and m), timed on a bounded sample of the
    same workload: the gridding over 1/8 and 1/4 of the sources and the
    interpolation over 1/8 and 1/4 of the nodes (seeded subsets), each
    extrapolated linearly to all, the FFT, multiplication and inverse FFT timed
    in full. Numpy runs these steps on one core."""
    import dataclasses
    from oracle import direct, nufft, kernel
    p = direct.prepare_workload(wl)
    rng = np.random.default_rng(11)
    Mq, N = p.y.shape[0], p.x.shape[0]
    t_grid, t_int, a = [], [], None
    for frac in (8, 4):
        sub = np.sort(rng.choice(Mq, Mq // frac, replace=False))
        ps = dataclasses.replace(p, y=p.y[sub], w=p.w[sub], g=p.g[sub])
        t1 = time.perf_counter()
        a = nufft.gridding(ps, m, window_name)
        t_grid.append((Mq // frac, time.perf_counter() - t1))
    t1 = time.perf_counter()
    bl = nufft.spectrum_b(p, a, m, window_name)
    d = kernel.full_coefficients(p.omega, p.C, p.n) * bl
    gg = nufft.nfft_grid(p, d, m, window_name)
    t_spec = time.perf_counter() - t1
    for frac in (8, 4):
        tg = np.sort(rng.choice(N, N // frac, replace=False))
        t1 = time.perf_counter()
        nufft.interpolate(p, gg, m, tg, window_name)
        t_int.append((N // frac, time.perf_counter() - t1))

    def extrap(pts, total):
        (n1, t1_), (n2, t2_) = pts
        slope = max((t2_ - t1_) / (n2 - n1), 0.0)
        return t2_ + slope * (total - n2)

    t_total = extrap(t_grid, Mq) + t_spec + extrap(t_int, N)
    sample_s = sum(t for _, t in t_grid) + t_spec + sum(t for _, t in t_int)
    cpu = host_cpu()
    return {"value": round(npts / t_total, 2), "unit": "pts/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle R3 (plain CPU NUFFT, {window_name} m={m}) on the same workload: "
                       f"gridding timed on 1/8 and 1/4 of the {Mq} sources "
                       f"({t_grid[0][1]:.2f}, {t_grid[1][1]:.2f} s) and interpolation on 1/8 and "
                       f"1/4 of the {N} nodes ({t_int[0][1]:.2f}, {t_int[1][1]:.2f} s), both "
                       f"extrapolated linearly to all, FFT + multiply + inverse FFT in full "
                       f"({t_spec:.2f} s); {sample_s:.1f} s of CPU work, estimated full solve "
                       f"{t_total:.1f} s; numpy runs these steps single-threaded"),
            "host": cpu, "seconds_per_solve": round(t_total, 2)}


def cpu_baseline_definition(wl, npts, n_src_sample=2048, n_tgt_sample=2048):
    """The oracle's definition route (R2: NDFT over every kept mode, blocked
    complex GEMM on the host BLAS with all its threads), timed on a seeded
    sample of sources and of nodes and scaled linearly (its cost is linear in
    M_q + N for a fixed mode set)."""
    import dataclasses
    from oracle import direct
    p = direct.prepare_workload(wl)
    rng = np.random.default_rng(12)
    Mq, N = p.y.shape[0], p.x.shape[0]
    ns, nt = min(n_src_sample, Mq), min(n_tgt_sample, N)
    sub = np.sort(rng.choice(Mq, ns, replace=False))
    ps = dataclasses.replace(p, y=p.y[sub], w=p.w[sub], g=p.g[sub])
    t1 = time.perf_counter()
    b = direct.ndft_b(ps)
    t_src = time.perf_counter() - t1
    tg = np.sort(rng.choice(N, nt, replace=False))
    t1 = time.perf_counter()
    direct.phi_ndft(p, tg, b=b)
    t_tgt = time.perf_counter() - t1
    t_total = t_src * Mq / ns + t_tgt * N / nt
    return {"value": round(npts / t_total, 2), "unit": "pts/s", "cores": blas_threads(),
            "kind": "oracle",
            "sample": (f"oracle definition route (NDFT over all kept modes, host BLAS) on "
                       f"{ns} of {Mq} sources ({t_src:.2f} s) and {nt} of {N} nodes "
                       f"({t_tgt:.2f} s), scaled linearly to the whole workload "
                       f"(estimated {t_total:.0f} s per solve)"),
            "host": host_cpu()}


def main():
    args = parse()
    for mode, fn in (("potential", potential), ("mix32", mix32), ("serve", serve)):
        if getattr(args, mode):
            if args.gpus != 1:
                print("bench.py: one GPU only", file=sys.stderr)
                sys.exit(2)
            fn(args)
            return
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (--gpus 1); multi-GPU runs are not "
              "part of it", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1305_3162_amd as slp
    from synth.workloads import make_workload

    if args.calib_copy_mb > 0:
        nel = args.calib_copy_mb * (1 << 20) // 4
        src_c = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst_c = torch.empty_like(src_c)
        for _ in range(3):
            dst_c.copy_(src_c)
        torch.cuda.synchronize()
        del src_c, dst_c
    prec = slp.FP64 if args.precision == "fp64" else slp.FP32
    window, m = resolve_window(args, slp, prec)
    kb = window == slp.WINDOW_KB
    wname = "kb" if kb else "gauss"
    wl = make_workload(args.workload, m)
    esz = 8 if prec == slp.FP64 else 4
    w, g = slp.expsum_sinc(wl.es_h, wl.es_r_lo, wl.es_r_hi, wl.es_tol)
    stream = torch.cuda.current_stream()
    targets = None
    if args.volume_targets:
        from synth import cube_volume_nodes
        if args.workload != "cube64":
            sys.exit("bench.py: --volume-targets needs the cube64 workload")
        targets = cube_volume_nodes(64)
    tune = None
    if args.autotune:
        tune = tuned_share(args, wl.nodes, wl.tris, wl.grid, m, w, g, wl.alpha, prec, wl.eta2,
                           window, targets)
    t1 = time.perf_counter()
    geom = slp.Geometry(wl.nodes, wl.tris, wl.grid, m, w, g, wl.alpha, prec, wl.eta2,
                        window=window, targets=targets,
                        seg_share=tune["seg_share"] if tune else 0,
                        reduce_cells=tune["reduce_cells"] if tune else 0)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t1
    near_cfg = None
    if args.near_tol is not None:
        t1 = time.perf_counter()
        eps = geom.near_radius(args.near_tol)
        storage = near_storage(args, slp, prec)
        geom.setup_near_field(eps, stream, storage)
        nf = geom.near_field_info()
        near_cfg = {"tol": args.near_tol, "eps": round(eps, 6), "pairs": nf["nnz"],
                    "stored": nf["stored"], "packed_columns": nf["packed"],
                    "values_stored_as": "fp64" if storage == slp.FP64 else "fp32",
                    "setup_s": round(time.perf_counter() - t1, 3),
                    "device_bytes": geom.info["device_bytes"]}
    iw_cfg = None
    if args.integrated:
        t1 = time.perf_counter()
        geom.setup_integrated_gridding(args.integrated, stream)
        iwi = geom.integrated_gridding_info()
        iw_cfg = {"order": iwi["order"], "window_integrals": iwi["nnz"], "stored": iwi["stored"],
                  "packed_columns": iwi["packed"], "setup_s": round(time.perf_counter() - t1, 3),
                  "device_bytes": slp.geom_get_info(geom.handle)["device_bytes"]}
    n_tgt = geom.info["n_targets"]
    geom_share, geom_segments = int(geom.info["seg_share"]), int(geom.info["n_segments"])
    geom_cells = int(geom.info["reduce_cells"])
    info = dict(geom.info)
    info["_n"] = [wl.grid[q] // wl.alpha for q in range(3)]
    info["_stored"] = 0 if near_cfg is None else near_cfg["stored"]
    info["_packed"] = False if near_cfg is None else near_cfg["packed_columns"]
    if near_cfg is not None:
        info["_near_esz"] = 8 if near_cfg["values_stored_as"] == "fp64" else 4
    info["_iw_stored"] = 0 if iw_cfg is None else iw_cfg["stored"]
    info["_iw_packed"] = False if iw_cfg is None else iw_cfg["packed_columns"]
    dens = torch.as_tensor(wl.dens, device="cuda")
    phi = torch.empty(n_tgt, dtype=torch.float64, device="cuda")
    nb = max(1, args.batch)
    if nb > 1:
        from synth import RandomSmoothMagnetisation, density_from_magnetisation
        dl = [dens] + [torch.as_tensor(density_from_magnetisation(
            wl.nodes, wl.tris, RandomSmoothMagnetisation(4000 + k, wl.nodes.min(0),
                                                         wl.nodes.max(0))), device="cuda")
            for k in range(1, nb)]
        pl = [phi] + [torch.empty_like(phi) for _ in range(1, nb)]
        hl = [geom.handle] * nb

    def step():
        if nb > 1:
            slp.eval_batched(hl, dl, pl, stream)
        else:
            geom.set_density(dens, stream)
            geom.eval(phi, stream)

    if args.graph:
        slp.set_graph(geom.handle, True)
    # timed region: K steps; the library records per-stage HIP events on the eval
    # stream for every 16th step (the event packets cost ~3 us each, so sampling
    # keeps them out of the throughput figure)
    ms_per_step, avg, cnt = timed_steps(torch, slp, geom, step, args.steps, args.warmup, stream)
    pts = (wl.n_src + n_tgt) * nb
    value = pts / (ms_per_step * 1e-3)
    if cnt == 0:           # graph replays record no stage events
        avg = {k: 0.0 for k in avg}
    dom = max(avg, key=avg.get)
    key = traffic_key(args.workload, args.precision, wname, m,
                      args.near_tol if near_cfg is not None else None, args.near_storage,
                      args.integrated)
    roofline = roofline_of(dom, avg, info, m, esz, nb, prec == slp.FP64, key, cnt)
    out_phi = phi.cpu().numpy()
    film_golden = (args.workload == "film512" and targets is None and near_cfg is None
                   and iw_cfg is None)
    rel_err, err_kind, err_extra = None, None, {}
    if film_golden:
        # stored oracle values: no oracle code runs for this error
        rel_err, n = golden_error(wl, geom, out_phi)
        err_kind = f"relative L2 over {n} stored oracle nodes (definition route)"
    geom.close()

    ref = None
    if not args.no_oracle and not film_golden:
        from oracle import direct
        p = direct.prepare(wl.nodes, wl.tris, wl.dens, wl.grid, wl.alpha, wl.es_h,
                           wl.es_r_lo, wl.es_r_hi, wl.es_tol, wl.eta2, targets=targets)
        ref = direct.phi_ndft(p)
        if near_cfg is None:
            rel_err = float(np.linalg.norm(out_phi - ref) / np.linalg.norm(ref))
            err_kind = "relative L2 over all targets (oracle definition route)"
        else:
            # the oracle's near-field sum on 8 seeded rows
            from oracle import nearfield as nfo
            rows = np.random.default_rng(7).choice(n_tgt, 8, replace=False)
            xs = (wl.nodes if targets is None else targets)[rows]
            rp_o, cols_o, _ = nfo.near_pairs(wl.nodes, wl.tris, xs, near_cfg["eps"])
            vals_o = nfo.near_values(p, wl.nodes, wl.tris, xs, rp_o, cols_o)
            gbar = nfo.element_mean_density(p, wl.tris.shape[0])
            near_o = np.add.reduceat(vals_o * gbar[cols_o], rp_o[:-1]) / nfo.FOUR_PI
            r_ref = ref[rows] + near_o
            d = out_phi[rows] - r_ref
            rel_err = float(np.linalg.norm(d) / np.linalg.norm(r_ref))
            err_kind = "relative L2 over 8 seeded rows (oracle smooth part + near-field sum)"
            err_extra = {"max_abs_err_over_max_abs_phi": float(np.abs(d).max()
                                                                / np.abs(ref).max())}
        if iw_cfg is not None:
            err_kind += ("; against the three-point definition, from which integrated-window "
                         "gridding differs by the three-point rule's quadrature error")

    extras = {}
    plain = (not args.no_extras and nb == 1 and near_cfg is None and iw_cfg is None
             and targets is None and not args.graph and not args.autotune)
    if plain and args.workload == "film512" and prec == slp.FP64:
        tf = time.perf_counter()
        # the film with the Gaussian window at the same gate, and in FP32
        wg, mg = slp.choose_cutoff(GATE["fp64"], slp.FP64, slp.WINDOW_GAUSS)
        extras["film_fp64_gaussian_same_gate"] = solve_line(
            args, slp, torch, make_workload("film512", mg), slp.FP64, wg, mg, 20, 3, "golden")
        w32, m32 = slp.choose_cutoff(GATE["fp32"], slp.FP32)
        extras["film_fp32"] = solve_line(args, slp, torch, make_workload("film512", m32),
                                         slp.FP32, w32, m32, 20, 3, "golden")
        wg32, mg32 = slp.choose_cutoff(GATE["fp32"], slp.FP32, slp.WINDOW_GAUSS)
        extras["film_fp32_gaussian"] = solve_line(args, slp, torch,
                                                  make_workload("film512", mg32), slp.FP32,
                                                  wg32, mg32, 20, 3, "golden")
        # the 64-cell cube (the previous default line) at both precisions
        cube = make_workload("cube64", m)
        extras["cube64_fp64"] = solve_line(args, slp, torch, cube, slp.FP64, window, m, 100, 10,
                                           "full")
        extras["cube64_fp64_gaussian_m8"] = solve_line(args, slp, torch,
                                                       make_workload("cube64", 8), slp.FP64,
                                                       slp.WINDOW_GAUSS, 8, 100, 10, "full")
        extras["cube64_fp32"] = solve_line(args, slp, torch, make_workload("cube64", m32),
                                           slp.FP32, w32, m32, 100, 10, "full")
        # batched: 64 densities on the cube in one launch; 32 icospheres in one call
        extras["batched_64_densities_cube64"] = {
            "fp64": batched_densities(args, slp, torch, cube, slp.FP64, window, m, 64, 5, 1),
            "fp32": batched_densities(args, slp, torch, make_workload("cube64", m32), slp.FP32,
                                      w32, m32, 64, 5, 1)}
        extras["multi_mesh_32_icospheres"] = {
            "fp64": multi_mesh(args, slp.FP64, window, m, 10, 2),
            "fp32": multi_mesh(args, slp.FP32, w32, m32, 10, 2)}
        extras["served_mix"] = served_mix(args, [0.5, 0.8, 0.95], args.requests, args.discard)
        extras["extras_wall_s"] = round(time.perf_counter() - tf, 1)

    cpu_baseline = None
    if not args.no_oracle and not args.no_cpu_baseline:
        if args.workload == "film512" and plain:
            cpu_baseline = cpu_baseline_r3(wl, m, wname, pts)
            extras["cpu_baseline_definition"] = cpu_baseline_definition(wl, pts)
        elif ref is not None:
            from oracle import direct
            reps, t_cpu = 0, 0.0
            while reps == 0 or t_cpu < 10.0:
                t1 = time.perf_counter()
                direct.phi_ndft(p)
                t_cpu += time.perf_counter() - t1
                reps += 1
            cpu_baseline = {"value": round(pts / (t_cpu / reps), 2), "unit": "pts/s",
                            "cores": blas_threads(), "kind": "oracle",
                            "sample": (f"oracle definition route (NDFT, host BLAS) over all "
                                       f"{wl.n_src} sources and {n_tgt} targets of the same "
                                       f"workload, {reps} solves in {t_cpu:.2f} s"
                                       + ("; near-field rows not included" if near_cfg else "")),
                            "host": host_cpu()}

    if args.workload in ("cube64", "film512"):
        wtext = workload_text(wl, n_tgt, window, m, targets)
    else:
        wtext = wl.name
    rec = {
        "metric": "SL-potential NUFFT (M+N) pts/s at stated rel err",
        "value": round(value, 1),
        "unit": "pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == slp.FP64 else "f32",
        "data": "synthetic",
        "config": {"workload": wtext, "m": m, "window": wname, "precision": args.precision,
                   "window_choice": ("as given" if args.m is not None else
                                     f"slp_choose_cutoff(tol={args.tol or GATE[args.precision]})"),
                   "points": pts, "densities_per_step": nb, "near_field": near_cfg,
                   "integrated_gridding": iw_cfg, "setup_s": round(t_setup, 3),
                   "gridding_split": {"seg_share": geom_share, "segments": geom_segments,
                                      "reduce_cells": geom_cells, "autotune": tune}},
        "rel_l2_err_vs_oracle": rel_err,
        "err_kind": err_kind,
        **err_extra,
        "stage_us": {k: round(v * 1e3, 3) for k, v in avg.items()},
        "roofline": roofline,
        "cpu_baseline": cpu_baseline,
        **extras,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
