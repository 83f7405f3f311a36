"""Benchmark of the matrix-free FE Kohn-Sham H.X on one MI355X.

A step is one full operator application Y = H X (local terms on every cell
plus the nonlocal projector term) of the 'mid' workload: periodic cube
L = 20 bohr, 16^3 cells, degree 6, 7 Gauss points, Gamma point, real FP64,
GGA field, 32 atoms x 4 projectors, 256 vectors (884,736 unique DoFs).
Inputs are resident in HBM before the timed region.

Printed (one JSON line): DoF*vectors/s over K timed steps, the roofline of
the dominant kernel (the local-operator kernel, timed separately with HIP
events on the stream it is launched on, per launch), and the CPU oracle's
rate on a bounded sample of the same workload (rank 0, N = 1 only).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec f64|f32|bf16]
                  [--workload mid|complex] [--no-cpu]

  python bench.py --filter   mixed-precision filter workload: the Mid operator
      with 512 vectors, filter degree 40, 3 outer passes of Lanczos bounds +
      filter + Rayleigh-Ritz per precision from the same seeds; one pass timed
      per precision; eigenvalue errors of the lowest 400 against the FP64 run.

  python bench.py --serve [--serve-run R] [--serve-runs K] [--requests 64]
      serving streams: requests with Poisson arrivals, each a random periodic
      system (cubic mesh 6^3..20^3 cells, p 5..8, 32..512 vectors, 8..64 atoms
      with 4 or 9 projectors, real or complex k) asking for one degree-20
      filter pass (FP32 inner steps); meshes resident, admission by HBM
      budget.  Per stream the arrival rate is 80% of the inverse mean service
      time of all its requests run alone; the same arrivals go through
      continuous batching in the library's request server (16 active; and
      with the admission work cap) and through its FIFO one-at-a-time mode;
      prints p50/p99 latency and throughput of each (median over the K
      streams) as one JSON line.
"""
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

METRIC = "H·X DoF·vectors/s FP64 vs FP32/BF16 filter at 1e-5 Ha; p50/p99 latency"
PEAK = {"f64": 78.6, "f32": 78.6, "bf16": 78.6}      # TFLOP/s, vector ALU (no packed FP32)
HBM_PEAK = 8000.0                                     # GB/s


def flops_per_cell_vec(np_, nq, cplx):
    """Eqn flopRealMF / flopComplexMF per cell per vector (even-odd counts)."""
    npo, nqo = np_ // 2, nq // 2
    lead = 2 * (npo * (nq + 2) + nqo * (np_ + 2)) * (np_ ** 2 + np_ * nq + nq ** 2) + 6 * nqo * nq ** 2 * (2 * nq + 5)
    return (lead + (40 if cplx else 34) * nq ** 3) * (2 if cplx else 1)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", default="f64", choices=["f64", "f32", "bf16"])
    ap.add_argument("--workload", default="mid", choices=["mid", "complex"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--nq-plus", type=int, default=0, choices=[0, 2],
                    help="quadrature n_q = n_p + this (2: the accurate rule)")
    ap.add_argument("--cpu-cells", type=int, default=0, help="0: every cell (whole H.X)")
    ap.add_argument("--filter", action="store_true")
    ap.add_argument("--filter-degree", type=int, default=40)
    ap.add_argument("--kpoints", action="store_true",
                    help="2x2x2 Monkhorst-Pack grid of the Mid system: batched vs separate H.X")
    ap.add_argument("--kpoint-nvec", type=int, default=64)
    ap.add_argument("--quad-study", action="store_true",
                    help="n_q = n_p, n_p + 2, n_p + 3 at FEOrder 8: H.X time ratios vs the flop model")
    ap.add_argument("--serve", action="store_true")
    ap.add_argument("--serve-run", type=int, default=0, help="first serving stream seed offset")
    ap.add_argument("--serve-runs", type=int, default=1, help="serving streams (each --requests long)")
    ap.add_argument("--serve-work-cap", type=float, default=2.5e8,
                    help="DoF x lanes per step past which the capped mode stops batching")
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--serve-budget-gb", type=float, default=150.0)
    ap.add_argument("--serve-degree", type=int, default=20)
    ap.add_argument("--serve-inner", default="f32", choices=["f64", "f32", "bf16"])
    return ap.parse_args()


def kernel_source_sha():
    """Hash of the local-operator kernel source (ties counter figures to the code)."""
    path = os.path.join(ROOT, "paper_2512_08571_amd", "csrc", "k_local_impl.h")
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def recorded_traffic(workload, prec, tile):
    """HBM bytes per k_local launch from the committed counter summary, or None.

    profiles/k_local_<workload>_<prec>_traffic.txt holds 'key: value' lines
    (per tile) written from two rocprofv3 --pmc runs of this script
    (FETCH_SIZE, then WRITE_SIZE), scaled by the counters' reading for a plain
    copy of known size in the same runs.  The figure is used only while the
    kernel source is the one it was measured on.
    """
    path = os.path.join(ROOT, "profiles", f"k_local_{workload}_{prec}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != kernel_source_sha():
        return None
    try:
        return int(float(kv[f"tile_{tile}_fetch_bytes_per_launch"]) + float(kv[f"tile_{tile}_write_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def make_block(torch, X, prec, cplx):
    t = torch.from_numpy(X).to("cuda:0")
    if prec == "f32":
        t = t.to(torch.complex64 if cplx else torch.float32)
    elif prec == "bf16":
        t = (torch.view_as_real(t) if cplx else t).to(torch.bfloat16).contiguous()
    return t


def host_cpu_model():
    """The host CPU's model name (from /proc/cpuinfo, as lscpu reports it)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(s, X, cells, min_s=10.0, max_s=30.0):
    """The oracle's cell-matrix route timed on the host cores.

    The whole H X of the workload (local cell matrices of every cell, or of a
    sample of 'cells' cells, plus the projector term when all cells are in),
    repeated until at least min_s seconds of CPU work (at most ~max_s).  Cell
    matrices and the projector matrix are built before the timed region.
    """
    from oracle import operator as op
    from oracle.mesh import Mesh as OMesh
    from paper_2512_08571_amd import inputs
    om = OMesh(s.lattice, s.ncell, s.degree, s.nq, s.kpoint)
    rng = np.random.default_rng(0)
    ncell = om.E if cells <= 0 or cells >= om.E else cells
    sample = np.arange(om.E) if ncell == om.E else np.sort(rng.choice(om.E, size=ncell, replace=False))
    pts = op.quad_points_of(om, sample).reshape(-1, 3)
    vl = np.zeros(om.E * om.nq ** 3)
    vg = np.zeros((om.E * om.nq ** 3, 3))
    idx = (sample[:, None] * om.nq ** 3 + np.arange(om.nq ** 3)[None, :]).reshape(-1)
    vl[idx] = inputs.eval_vloc(s, pts)
    if s.gga_coef is not None:
        vg[idx] = inputs.eval_vgga(s, pts)
    He = op.element_matrices(om, vl, vg, sample)          # set-up, not timed
    P = h = None
    if ncell == om.E and s.projectors:
        P, h = op.projector_matrix(om, inputs.positions_array(s), s.projectors)
    reps, t0 = 0, time.perf_counter()
    while True:
        op.apply_cm(om, vl, vg, X, P, h, cells=sample, He=He)
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= min_s or dt * (reps + 1) / reps > max_s:
            break
    dofvec = reps * len(sample) * s.degree ** 3 * X.shape[1]
    blas = "unknown"
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        cores = max([i.get("num_threads", 1) for i in info] + [1])
        blas = ", ".join(f"{i.get('internal_api')} {i.get('version')} ({i.get('num_threads')} threads)"
                         for i in info if i.get("user_api") == "blas") or blas
    except Exception:
        cores = os.cpu_count()
    what = "all" if ncell == om.E else f"{len(sample)} sampled"
    return {"value": dofvec / dt, "unit": "DoF*vectors/s", "cores": int(cores), "kind": "oracle",
            "host_cpu": host_cpu_model(), "host_logical_cpus": os.cpu_count(), "blas": blas,
            "sample": (f"oracle cell-matrix H.X ({what} of {om.E} cells x {X.shape[1]} vectors"
                       f"{', with the projector term' if P is not None else ', local terms only'}), "
                       f"{reps} repetitions, {dt:.1f} s timed; cell and projector matrices built "
                       f"before timing; DoF*vectors counted as p^3 unique DoFs per cell")}


def subspace_sin(U, V, d):
    """sin of the largest principal angle between span(U) and span(V) in the
    inner product <x, y> = x^H diag(d) y, for D-orthonormal U and V (device
    blocks [m, k]): the D-norm of U - V (V^H D U)."""
    import torch
    G = V.conj().T @ (d[:, None] * U)
    R = U - V @ G
    S = R.conj().T @ (d[:, None] * R)
    ev = torch.linalg.eigvalsh(0.5 * (S + S.conj().T))
    return float(ev.clamp(min=0).max().sqrt())


def filter_golden():
    """The oracle's Ritz values of the filter workload (tests/golden/filter_eigs.npz), or None."""
    path = os.path.join(ROOT, "tests", "golden", "filter_eigs.npz")
    if not os.path.exists(path):
        return None
    g = np.load(path)
    return g["ritz"], int(g["degree"]), int(g["outer"])


def filter_bench(a):
    """Filter workload: FP64 vs FP32 / BF16 inner steps (one JSON line)."""
    import torch
    from paper_2512_08571_amd import fehx, inputs

    s = inputs.make_system("filter")
    m = fehx.Mesh(s.lattice, s.ncell, s.degree, s.nq, s.kpoint, device=0)
    pts = m.quad_points()
    m.set_potential(inputs.eval_vloc(s, pts), inputs.eval_vgga(s, pts))
    m.set_projectors(inputs.positions_array(s), s.projectors)
    X0 = torch.from_numpy(inputs.make_vectors(s, seed_offset=0)).cuda()
    v0 = torch.from_numpy(inputs.lanczos_start(s)).cuda()
    deg, nv = a.filter_degree, s.nvec
    keep = min(400, nv)
    res = {}
    for prec in ("f64", "f32", "bf16"):
        m.autotune(prec, nv, kind=1, reps=2)
        # one pass timed on the start block with its Rayleigh-Ritz values
        X = X0.clone()
        ritz = torch.empty(nv, dtype=torch.float64, device="cuda")
        m.rayleigh_ritz(X, ritz)
        theta, beta = m.lanczos(v0, 10)
        lmin, lmax = theta.min(), theta.max() + abs(beta)
        lT = lmin + 0.5 * (6 * np.pi ** 2 * nv / s.volume) ** (2.0 / 3.0)
        Xt = X.clone()
        m.cheb_filter(Xt, ritz, deg, lmin, lT, lmax, inner=prec)      # warm-up
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 3
        e0.record()
        for _ in range(reps):
            Xt.copy_(X)
            m.cheb_filter(Xt, ritz, deg, lmin, lT, lmax, inner=prec)
        e1.record()
        torch.cuda.synchronize()
        ms_pass = e0.elapsed_time(e1) / reps
        # the same pass captured once as a HIP graph and replayed
        g = m.filter_graph(Xt, ritz, deg, lmin, lT, lmax, inner=prec)
        Xt.copy_(X)
        g.launch()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            Xt.copy_(X)
            g.launch()
        e1.record()
        torch.cuda.synchronize()
        ms_graph = e0.elapsed_time(e1) / reps
        g.close()
        del Xt
        # the eigensolver procedure from the same seeds
        X = X0.clone()
        t0 = time.perf_counter()
        lam, bounds = m.chfsi(X, v0, outer=3, degree=deg, inner=prec)
        res[prec] = dict(ms_pass=ms_pass, ms_graph=ms_graph, lam=lam, chfsi_s=time.perf_counter() - t0,
                         X=X[:, :keep].contiguous())
        del X
    out = {"metric": "filter pass time and eigenvalue error, FP32/BF16 vs FP64 inner steps",
           "value": res["f64"]["ms_pass"] / res["f32"]["ms_pass"], "unit": "speedup FP32 vs FP64",
           "higher_is_better": True, "n_gpus": 1, "dtype": "f64/f32/bf16", "data": "synthetic",
           "config": {"workload": f"filter: Mid operator (16^3 cells, p=6, GGA, 32 atoms x 4 projectors), "
                                  f"{nv} vectors, degree {deg}, 3 outer passes", "ndofs": m.ndofs}}
    gold = filter_golden()
    if gold is not None and (gold[1], gold[2]) != (deg, 3):
        gold = None
    dvec = torch.from_numpy(m.lumped_mass()).cuda()
    for prec in ("f64", "f32", "bf16"):
        r = res[prec]
        d = np.abs(r["lam"][:keep] - res["f64"]["lam"][:keep])
        o = {"ms_per_pass": round(r["ms_pass"], 3), "ms_per_pass_graph_replay": round(r["ms_graph"], 3),
             "speedup_vs_f64": round(res["f64"]["ms_pass"] / r["ms_pass"], 3),
             "max_abs_dlambda_lowest_%d_vs_gpu_f64_ha" % keep: float(d.max()),
             "subspace_sin_max_lowest_%d_vs_gpu_f64" % keep: subspace_sin(r["X"], res["f64"]["X"], dvec),
             "dofvec_per_s_in_pass": m.ndofs * nv * deg / (r["ms_pass"] * 1e-3),
             "chfsi_s": round(r["chfsi_s"], 2), "lowest_eigenvalue": float(r["lam"][0])}
        if gold is not None:
            dg = np.abs(r["lam"][:keep] - gold[0][:keep])
            o["max_abs_dlambda_lowest_%d_vs_oracle_f64_ha" % keep] = float(dg.max())
            o["gate_1e-5_ha"] = bool(dg.max() <= 1e-5)
        out[prec] = o
    out["reference"] = ("oracle FP64 Ritz values, tests/golden/filter_eigs.npz (same procedure and seeds)"
                        if gold is not None else "GPU FP64 run only (no oracle golden for this degree)")
    out["gap_400_401_ha"] = float(res["f64"]["lam"][keep] - res["f64"]["lam"][keep - 1]) if nv > keep else None
    print(json.dumps(out))


def kpoint_bench(a):
    """Eight k-points (2x2x2 Monkhorst-Pack grid) of the Mid system: the eight
    complex H.X per step as one fe_batch_apply (one batched launch per colour
    phase) against eight separate fe_apply_H calls (one JSON line)."""
    import dataclasses as dc
    import torch
    from paper_2512_08571_amd import fehx, inputs

    base = inputs.make_system("mid")
    Ld = np.diag(base.lattice)
    u = [-0.25, 0.25]
    ks = [2 * np.pi * np.array([x, y, z]) / Ld for x in u for y in u for z in u]
    nv = a.kpoint_nvec
    meshes = []
    vl = vg = None
    for k in ks:
        s = dc.replace(base, kpoint=k)
        m = fehx.Mesh(s.lattice, s.ncell, s.degree, s.nq, s.kpoint, device=0)
        if vl is None:
            pts = m.quad_points()
            vl, vg = inputs.eval_vloc(s, pts), inputs.eval_vgga(s, pts)
        m.set_potential(vl, vg)
        m.set_projectors(inputs.positions_array(s), s.projectors)
        meshes.append(m)
    g = torch.Generator(device="cuda").manual_seed(5)
    Xs = [torch.complex(torch.rand(base.ndofs, nv, dtype=torch.float64, device="cuda", generator=g) - 0.5,
                        torch.rand(base.ndofs, nv, dtype=torch.float64, device="cuda", generator=g) - 0.5)
          for _ in ks]
    Ys = [torch.empty_like(x) for x in Xs]
    meshes[0].autotune("f64", nv)
    vt = meshes[0].get_tile("f64")
    for m in meshes[1:]:
        m.set_tile("f64", vt)
    stream = torch.cuda.current_stream()

    def separate():
        for m, x, y in zip(meshes, Xs, Ys):
            m.apply(x, y, "f64", stream=stream)

    def batched():
        fehx.batch_apply(meshes, Xs, Ys, "f64", stream=stream)

    res = {}
    for name, f in (("separate", separate), ("batched", batched)):
        for _ in range(a.warmup):
            f()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(a.steps):
            f()
        e1.record(stream)
        torch.cuda.synchronize()
        res[name] = e0.elapsed_time(e1) / a.steps
    dofvec = base.ndofs * nv * len(ks)
    out = {"metric": "H.X DoF*vectors/s over a k-point grid, batched launch", "unit": "DoF*vectors/s",
           "value": dofvec / (res["batched"] * 1e-3), "higher_is_better": True, "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "dtype": "f64", "data": "synthetic",
           "ms_per_step_batched": round(res["batched"], 3), "ms_per_step_separate": round(res["separate"], 3),
           "separate_dofvec_per_s": dofvec / (res["separate"] * 1e-3), "tile": vt,
           "config": {"workload": (f"kpoints: Mid system (16^3 cells, p=6, nq=7, GGA, 32 atoms x 4 projectors) "
                                   f"at the 8 points of a 2x2x2 Monkhorst-Pack grid, {nv} complex vectors each"),
                      "ndofs": base.ndofs, "nvec_per_k": nv, "kpoints": len(ks)}}
    print(json.dumps(out))


def quad_study(a):
    """Quadrature-rule cost at FEOrder 8 (the paper's remark in Sec. 5.3):
    FP64 H X (local operator, GGA, no projectors) of a periodic 12^3-cell box,
    p = 8, 256 vectors, with n_q = n_p, n_p + 2 and n_p + 3; times per H X
    with the autotuned tile and the ratios next to the flop model's."""
    import torch
    from paper_2512_08571_amd import fehx, inputs

    p, nv, L = 8, 256, 15.0
    res = {}
    for dq in (0, 2, 3):
        s = inputs.make_custom(np.eye(3) * L, (12, 12, 12), p, p + 1 + dq, nvec=nv, seed=41, ngauss=6)
        m = fehx.Mesh(s.lattice, s.ncell, s.degree, s.nq, s.kpoint, device=0)
        pts = m.quad_points()
        m.set_potential(inputs.eval_vloc(s, pts), inputs.eval_vgga(s, pts))
        g = torch.Generator(device="cuda").manual_seed(3)
        X = torch.rand(m.ndofs, nv, dtype=torch.float64, device="cuda", generator=g) - 0.5
        Y = torch.empty_like(X)
        tile, _ = m.autotune("f64", nv, reps=2)
        for _ in range(a.warmup):
            m.apply(X, Y)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(a.steps):
            m.apply(X, Y)
        e1.record()
        torch.cuda.synchronize()
        res[dq] = dict(ms=e0.elapsed_time(e1) / a.steps, tile=tile,
                       flop=flops_per_cell_vec(p + 1, p + 1 + dq, False))
        del X, Y, m
        torch.cuda.empty_cache()
    out = {"metric": "H.X time ratio between quadrature rules, FEOrder 8", "n_gpus": 1, "dtype": "f64",
           "data": "synthetic", "steps": a.steps, "warmup": a.warmup,
           "config": {"workload": f"quadrature study: periodic cube L={L:g} bohr, 12^3 cells, p={p}, GGA, "
                                  f"{nv} real vectors, FP64, local operator"},
           "ms_per_hx": {f"nq=np+{dq}": round(r["ms"], 4) for dq, r in res.items()},
           "tiles": {f"nq=np+{dq}": r["tile"] for dq, r in res.items()},
           "ratio_np2_over_np": {"measured": round(res[2]["ms"] / res[0]["ms"], 3),
                                 "flop_model": round(res[2]["flop"] / res[0]["flop"], 3)},
           "ratio_np3_over_np2": {"measured": round(res[3]["ms"] / res[2]["ms"], 3),
                                  "flop_model": round(res[3]["flop"] / res[2]["flop"], 3)}}
    print(json.dumps(out))


def serve_stream(srv, reqs, arrivals, block, submit, x_cap=80 << 30):
    """Feed the requests to a server at their arrival times; latency per request
    (completion - arrival, s) and the makespan (first arrival to last completion)."""
    import numpy as np
    live, lat, done_ids = {}, [None] * len(reqs), set()
    live_bytes, nxt = 0, 0
    t0 = time.perf_counter()
    while len(done_ids) < len(reqs):
        now = time.perf_counter() - t0
        while nxt < len(reqs) and arrivals[nxt] <= now:
            r = reqs[nxt]
            nbytes = r["s"].ndofs * r["s"].nvec * (16 if r["s"].is_complex else 8)
            if live and live_bytes + nbytes > x_cap:
                break                        # the caller waits for blocks to free up
            X = block(r)
            live[nxt] = (submit(srv, r, X), X, nbytes)
            live_bytes += nbytes
            nxt += 1
        active, queued = srv.progress(block=False)
        for i in list(live):
            rid, X, nbytes = live[i]
            st, (ts, ta, td), err = srv.status(rid)
            if st >= 2:
                if st != 2:
                    raise RuntimeError(f"request {i} failed with status {err}")
                lat[i] = td - (t0 + arrivals[i])
                done_ids.add(i)
                srv.release(rid)
                del live[i]
                live_bytes -= nbytes
        if nxt < len(reqs) and not live:
            time.sleep(max(0.0, min(0.002, arrivals[nxt] - (time.perf_counter() - t0))))
        elif active and nxt >= len(reqs):
            srv.progress(block=True)
    return np.array(lat), time.perf_counter() - t0


def serve(a):
    """The serving stream through the library's request server (one JSON line).

    Per run: 64 random systems (inputs.make_serving_stream); every request's
    service time alone sets the Poisson arrival rate (80% load on the whole
    stream's mean); the same arrivals then go through continuous batching
    (16 active) and through the FIFO baseline (one request at a time, in
    arrival order) of the same server."""
    import torch
    from paper_2512_08571_amd import fehx, inputs

    def block(r):
        s = r["s"]
        gen = torch.Generator(device="cuda").manual_seed(s.seed + 1)
        X = torch.rand(s.ndofs, s.nvec, dtype=r["dt"], device="cuda", generator=gen)
        return X.mul_(2).sub_(1 + (1j if s.is_complex else 0))

    def submit(srv, r, X):
        return srv.submit_filter(r["m"], X, r["lam"], a.serve_degree, *r["bounds"], inner=a.serve_inner)

    budget = int(a.serve_budget_gb * (1 << 30))
    runs, tuned = [], {}
    for run in range(a.serve_run, a.serve_run + a.serve_runs):
        print(f"serving run {run}: setup", file=sys.stderr, flush=True)
        systems = inputs.make_serving_stream(run, a.requests)
        t_setup = time.perf_counter()
        reqs = []
        for s in systems:
            m = fehx.Mesh(s.lattice, s.ncell, s.degree, s.nq, s.kpoint, device=0)
            v, g = inputs.eval_serving_fields(s, m.quad_points())
            m.set_potential(v, g)
            m.set_projectors(inputs.positions_array(s), s.projectors)
            cls = (s.degree, s.is_complex)
            if cls not in tuned:            # one autotune per launch class (filter steps)
                tuned[cls] = m.autotune(a.serve_inner, s.nvec, kind=1, reps=2)[0]
            m.set_tile(a.serve_inner, tuned[cls], kind=1)
            gen = torch.Generator(device="cuda").manual_seed(s.seed)
            dt = torch.complex128 if s.is_complex else torch.float64
            v0 = torch.rand(s.ndofs, dtype=dt, device="cuda", generator=gen)
            theta, beta = m.lanczos(v0, 10)
            del v0
            lmin, lmax = theta.min(), theta.max() + abs(beta)
            lT = lmin + 0.5 * (6 * np.pi ** 2 * s.nvec / s.volume) ** (2.0 / 3.0)
            lT = min(lT, lmin + 0.5 * (lmax - lmin))
            lam = torch.linspace(lmin, lT, s.nvec, dtype=torch.float64, device="cuda")
            reqs.append(dict(s=s, m=m, lam=lam, bounds=(lmin, lT, lmax), dt=dt))
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t_setup
        # every request alone: its service time (the arrival rate comes from their mean)
        print(f"serving run {run}: service times alone", file=sys.stderr, flush=True)
        srv = fehx.Server(hbm_budget=budget, max_active=1)
        alone = []
        for r in reqs:
            X = block(r)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rid = submit(srv, r, X)
            srv.drain()
            alone.append(time.perf_counter() - t0)
            srv.release(rid)
            del X
        srv.close()
        mean_alone = float(np.mean(alone))
        rng = np.random.default_rng(inputs.SERVE_SEED0 + run + 1000)
        arrivals = np.cumsum(rng.exponential(mean_alone / 0.8, len(reqs)))
        res = {"run": run, "setup_s": round(t_setup, 2), "mean_alone_ms": mean_alone * 1e3,
               "arrival_rate_per_s": 0.8 / mean_alone, "arrival_window_s": float(arrivals[-1])}
        dofvec = sum(r["s"].ndofs * r["s"].nvec * a.serve_degree for r in reqs)
        for mode, active, cap in (("batching", 16, 0), ("capped", 16, a.serve_work_cap), ("fifo", 1, 0)):
            print(f"serving run {run}: {mode} stream", file=sys.stderr, flush=True)
            srv = fehx.Server(hbm_budget=budget, max_active=active)
            srv.set_work_cap(cap)
            lat, makespan = serve_stream(srv, reqs, arrivals, block, submit)
            ticks, held = srv.stats()
            allocs, frees, idle = srv.pool_stats()
            srv.close()
            lat_ms = lat * 1e3
            res[mode] = {"p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
                         "mean_ms": float(lat_ms.mean()), "makespan_s": makespan,
                         "throughput_dofvec_per_s": dofvec / makespan, "ticks": ticks,
                         "held_gb": held / 2 ** 30, "workspace_allocs": allocs, "workspace_frees": frees}
        runs.append(res)
        print(f"serving run {run}: p50 batching {res['batching']['p50_ms']:.0f} ms, capped "
              f"{res['capped']['p50_ms']:.0f} ms, fifo {res['fifo']['p50_ms']:.0f} ms", file=sys.stderr, flush=True)
        for r in reqs:
            r["m"].close()
        del reqs
        torch.cuda.empty_cache()

    def med(mode, key):
        return float(np.median([r[mode][key] for r in runs]))
    summary = {mode: {k: med(mode, k) for k in ("p50_ms", "p99_ms", "throughput_dofvec_per_s")}
               for mode in ("batching", "capped", "fifo")}
    out = {"metric": "serving p50/p99 latency, degree-%d filter requests" % a.serve_degree,
           "value": summary["batching"]["p50_ms"], "unit": "ms", "higher_is_better": False,
           "p50_ms": summary["batching"]["p50_ms"], "p99_ms": summary["batching"]["p99_ms"],
           "throughput_dofvec_per_s": summary["batching"]["throughput_dofvec_per_s"],
           "capped": summary["capped"], "fifo": summary["fifo"], "work_cap_dofvec": a.serve_work_cap,
           "beats_fifo": {mode: {k: (summary[mode][k] < summary["fifo"][k]) if k != "throughput_dofvec_per_s"
                                 else (summary[mode][k] > summary["fifo"][k])
                                 for k in ("p50_ms", "p99_ms", "throughput_dofvec_per_s")}
                          for mode in ("batching", "capped")},
           "runs": runs, "requests_per_run": a.requests,
           "dtype": a.serve_inner, "data": "synthetic", "n_gpus": 1,
           "config": {"workload": f"serving streams runs {a.serve_run}..{a.serve_run + a.serve_runs - 1}: "
                                  f"{a.requests} random periodic systems each, 6^3..20^3 cells, p 5..8, "
                                  f"32..512 vectors, 8..64 atoms x 4/9 projectors, real/complex k, Poisson "
                                  f"arrivals at 80% of the stream's mean service time alone",
                      "budget_gb": a.serve_budget_gb, "tiles": {f"p{k[0]}{'c' if k[1] else 'r'}": v
                                                                 for k, v in tuned.items()},
                      "statistic": "median over runs"}}
    print(json.dumps(out))


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if a.serve:
        serve(a)
        return
    if a.quad_study:
        quad_study(a)
        return
    if a.filter:
        filter_bench(a)
        return
    if a.kpoints:
        kpoint_bench(a)
        return
    import torch
    from paper_2512_08571_amd import fehx, inputs

    s = inputs.make_system(a.workload)
    if a.nq_plus:
        s = dataclasses.replace(s, nq=s.degree + 1 + a.nq_plus)
    cplx = s.is_complex
    m = fehx.Mesh(s.lattice, s.ncell, s.degree, s.nq, s.kpoint, device=0)
    m_loc = fehx.Mesh(s.lattice, s.ncell, s.degree, s.nq, s.kpoint, device=0)
    pts = m.quad_points()
    vl, vg = inputs.eval_vloc(s, pts), inputs.eval_vgga(s, pts)
    for mm in (m, m_loc):
        mm.set_potential(vl, vg)
    m.set_projectors(inputs.positions_array(s), s.projectors)
    nv = s.nvec
    if a.workload == "complex":
        # 16 seeded columns tiled on the device to the full block (38.8 GB in
        # FP64): timing only needs the shape
        base = torch.from_numpy(inputs.make_vectors(s, cols=range(16))).to("cuda:0")
        Xd = base.repeat(1, nv // 16)
        del base
        if a.prec == "f32":
            Xd = Xd.to(torch.complex64)
        elif a.prec == "bf16":
            Xd = torch.view_as_real(Xd).to(torch.bfloat16).contiguous()
        X = None
    else:
        X = inputs.make_vectors(s)
        Xd = make_block(torch, X, a.prec, cplx)
    Yd = torch.empty_like(Xd)
    stream = torch.cuda.current_stream()
    # launch shape from the library's autotuner (untimed set-up), same on both meshes
    tile, tile_ms = m.autotune(a.prec, nv, kind=0, reps=2)
    m_loc.set_tile(a.prec, tile)
    # a plain copy of known size: the reference reading for the HBM byte counters
    Yd.copy_(Xd)
    torch.cuda.synchronize()
    for _ in range(a.warmup):
        m.apply(Xd, Yd, a.prec, stream)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(a.steps):
        m.apply(Xd, Yd, a.prec, stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / a.steps
    dofvec = m.ndofs * nv
    value = dofvec / (ms * 1e-3)

    # dominant kernel: the local operator alone (same launches, no projectors)
    for _ in range(2):
        m_loc.apply(Xd, Yd, a.prec, stream)
    torch.cuda.synchronize()
    reps = max(5, a.steps)
    ev0.record(stream)
    for _ in range(reps):
        m_loc.apply(Xd, Yd, a.prec, stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    nc = s.ncell
    nphase = (3 if nc[0] % 2 else 2) * (3 if nc[1] % 2 else 2)
    ms_launch = ev0.elapsed_time(ev1) / (reps * nphase)
    fl = flops_per_cell_vec(s.degree + 1, s.nq, cplx) * m.ncells * nv / nphase
    achieved = fl / (ms_launch * 1e-3) / 1e12
    traffic = recorded_traffic(a.workload, a.prec, tile) if not a.nq_plus else None
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK[a.prec], "unit": "TFLOP/s",
            "frac": round(achieved / PEAK[a.prec], 4), "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "algorithmic_bytes_per_launch": dofvec * (16 if a.prec == "f64" else 8 if a.prec == "f32" else 4)
                                            * (2 if cplx else 1) // nphase,
            "kernel": "k_local", "launch_ms": round(ms_launch, 4),
            "algorithmic_flop_per_launch": fl,
            "hbm_gbs_algorithmic": round(dofvec * (16 if a.prec == "f64" else 8 if a.prec == "f32" else 4)
                                         * (2 if cplx else 1) / nphase / (ms_launch * 1e-3) / 1e9, 1)}
    out = {"metric": METRIC, "value": value, "unit": "DoF*vectors/s", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": a.prec, "data": "synthetic",
           "config": {"workload": (f"{a.workload}: periodic cube L={s.lattice[0][0]:g} bohr, {nc[0]}^3 cells, "
                                   f"p={s.degree}, nq={s.nq}, {'complex Bloch' if cplx else 'real Gamma'}, "
                                   f"GGA, {len(s.atoms)} atoms x {len(s.projectors) // max(len(s.atoms), 1)} "
                                   f"projectors, nvec={nv}"),
                      "ndofs": m.ndofs, "nvec": nv, "precision": a.prec, "wall_s": round(wall, 3),
                      "tile": tile, "tile_ms": {str(k): round(v, 4) for k, v in tile_ms.items()},
                      "kernel_source_sha256": kernel_source_sha()},
           "roofline": roof}
    if not a.no_cpu and a.workload == "mid" and not a.nq_plus:
        del Xd, Yd
        out["cpu_baseline"] = cpu_baseline(s, X, a.cpu_cells)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
