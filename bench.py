"""Benchmark of the FE assembly + Jacobi-PCG hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload hex128]

A step is one pass of the whole hot path over the 128^3 HEX08 workload
(2,097,152 elements, shuffled numbering, jitter 15 %): momentum assembly
(M/dt + C + K and 3 RHS) and pressure-Laplacian assembly into CSR,
symmetric Dirichlet elimination, then exactly 200 Jacobi-PCG iterations.
Mesh preprocessing/upload is one-time and outside the timed region; the
fields are resident in HBM before timing starts.

Prints one JSON line: value = elements per second of the whole step (Melem/s),
plus the SpMV roofline (HEX08 SpMV is the dominant kernel: 200 launches per
step) measured with HIP events on the library's stream, and the CPU oracle
timed on a bounded sample of the same recipe (one thread and every thread).
After the timed step, the same run measures the metric's second half and the
large single mesh, each outside the timed region:
  serving: the first 400 requests of the serving stream (HEX08 cubes of side
           8..96, log-uniform; momentum + Poisson assembly + PCG to a true
           relative residual of 1e-8), sequential FP64 against the batching
           server, saturated and at 0.8x the sequential capacity;
  cfg4:    256^3 HEX08 with 5 species: 8 equations assembled, and the Poisson
           solve to 1e-8 by FP64 PCG and by FP32 PCG in FP64 refinement.
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

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6    # MI355X dense FP64 vector
FP32_PEAK_TFLOPS = 157.3   # MI355X dense FP32 vector
CG_ITERS = 200


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def spmv_bytes(nnz, n):
    # values 8 + colidx 4 per entry; rowptr 4 + x 8 + y 8 per row
    return 12 * nnz + 20 * n


def measured_valu(workload):
    """FP64/FP32 flops per element of the assembly kernels from the committed
    VALU-counter summary, or None once the assembly sources have changed since
    the counters were taken (or for another workload)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "assembly_hex128.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    kv = {}
    for ln in text.splitlines():
        ln = ln.strip()
        if ":" in ln:
            k, v = ln.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("valu_workload") != workload:
        return None
    h = hashlib.sha256()
    for rel in ("asm_kernels.hip", "internal.h", "plan.cpp", "rowplan.cpp"):
        with open(os.path.join(ROOT, "paper_2107_11541_amd", "csrc", rel), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != kv.get("valu_source_sha256"):
        return None
    keys = ("momentum_fp64_flops_per_element", "poisson_fp64_flops_per_element",
            "mixed_momentum_fp64_flops_per_element", "mixed_momentum_fp32_flops_per_element",
            "momentum_hbm_bytes_per_operator", "poisson_hbm_bytes_per_operator", "residual_fp64_flops_per_element")
    return {k: float(kv[k]) for k in keys if k in kv}


def assembly_roofline(workload, E, ms_mom, ms_poi, ms_mix):
    """Assembly against both rooflines: FLOP rates against the FP64 / FP32
    vector peaks and real HBM rates against 8 TB/s, from the counted flops
    per element and HBM bytes per operator and this run's assembly times
    (None when the counters do not describe the kernels as built)."""
    f = measured_valu(workload)
    if f is None:
        return None
    def rate(flops, ms):
        return flops * E / (ms * 1e-3) / 1e12
    mom = rate(f["momentum_fp64_flops_per_element"], ms_mom)
    poi = rate(f["poisson_fp64_flops_per_element"], ms_poi)
    m64 = rate(f["mixed_momentum_fp64_flops_per_element"], ms_mix)
    m32 = rate(f["mixed_momentum_fp32_flops_per_element"], ms_mix)
    return {"unit": "TFLOP/s", "fp64_peak": FP64_PEAK_TFLOPS, "fp32_peak": FP32_PEAK_TFLOPS,
            "counted": f,
            "momentum_fp64": mom, "momentum_fp64_frac": mom / FP64_PEAK_TFLOPS,
            "poisson_fp64": poi, "poisson_fp64_frac": poi / FP64_PEAK_TFLOPS,
            "mixed_momentum_fp64": m64, "mixed_momentum_fp32": m32,
            "mixed_momentum_frac": m64 / FP64_PEAK_TFLOPS + m32 / FP32_PEAK_TFLOPS,
            "hbm_unit": "GB/s", "hbm_peak": HBM_PEAK_GBS,
            "momentum_hbm_real": f["momentum_hbm_bytes_per_operator"] / (ms_mom * 1e-3) / 1e9,
            "momentum_hbm_frac": f["momentum_hbm_bytes_per_operator"] / (ms_mom * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "poisson_hbm_real": f["poisson_hbm_bytes_per_operator"] / (ms_poi * 1e-3) / 1e9,
            "poisson_hbm_frac": f["poisson_hbm_bytes_per_operator"] / (ms_poi * 1e-3) / 1e9 / HBM_PEAK_GBS}


def momentum_bytes(nnz, n, conn_entries):
    # coords 24 + u 24 + rho 8 + mu 8 per node, 4 per connectivity entry
    # (nen per element), values 8 per entry, rhs 24 per node (written once)
    return n * 64 + 4 * conn_entries + nnz * 8 + n * 24


def poisson_bytes(nnz, n, conn_entries):
    return n * 56 + 4 * conn_entries + nnz * 8 + n * 8


def measured_traffic(workload, kernel):
    """HBM bytes per launch of the dominant kernel from the committed PMC summary
    of this workload (profiles/<kernel>_<workload>.md).

    The summary records a hash of the solver kernel sources; once they have
    changed the counters describe another kernel and the figure is dropped
    (None), as it is for any workload the counters were not taken on.
    """
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    kv = {}
    for ln in text.splitlines():
        ln = ln.strip()
        if ":" in ln and ln.split(":", 1)[0] in ("traffic_kernel", "traffic_workload", "traffic_bytes_per_launch",
                                               "source_sha256"):
            k, v = ln.split(":", 1)
            kv[k] = v.strip()
    if kv.get("traffic_workload") != workload or kv.get("traffic_kernel") != kernel or \
            "traffic_bytes_per_launch" not in kv:
        return None
    h = hashlib.sha256()
    for rel in ("solver_kernels.hip", "internal.h"):
        with open(os.path.join(ROOT, "paper_2107_11541_amd", "csrc", rel), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != kv.get("source_sha256"):
        return None
    return float(kv["traffic_bytes_per_launch"])


def roofline_entry(workload, algo_bytes, avg_us, launches, symmetric):
    """The dominant kernel against the HBM roofline: achieved = its
    algorithmic bytes per launch (those of the CSR product it computes) over
    its average launch time; beside it the real HBM rate, the counted bytes
    per launch over the same time, while the counters describe the kernel as
    built (else null).  symmetric: the PCG ran the symmetric SpMV."""
    kernel = "k_cg_spmv_sym" if symmetric else "k_cg_spmv_pq"
    achieved = algo_bytes / (avg_us * 1e-6) / 1e9
    traffic = measured_traffic(workload, kernel)
    real = traffic / (avg_us * 1e-6) / 1e9 if traffic else None
    label = ("k_cg_spmv_sym (CSR SpMV, in-block symmetric pairs read once, fused with p.Ap)" if symmetric
             else "k_cg_spmv_pq (CSR SpMV fused with p.Ap)")
    return {"bound": "hbm", "kernel": label,
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic, "real_hbm_gbs": real, "real_frac": real / HBM_PEAK_GBS if real else None,
            "algorithmic_bytes_per_launch": algo_bytes, "avg_launch_us": avg_us, "launches": launches}


def make_workload(name):
    import meshgen
    if name == "hex128":
        return meshgen.cfg1(128), "hex08-128^3-shuffled-jitter15: momentum+Poisson assembly, Dirichlet, 200 PCG"
    if name == "hex64":
        return meshgen.cfg1(64), "hex08-64^3-shuffled-jitter15: momentum+Poisson assembly, Dirichlet, 200 PCG"
    if name == "tet128":
        return meshgen.cfg2(128), "tet04-6x128^3-flame: momentum+Poisson assembly, Dirichlet, 200 PCG"
    if name == "hybrid128":
        return meshgen.hybrid(128), ("hybrid-128^3-flame (prism | hex | pyramid-tet transition | tet slabs): "
                                     "momentum+Poisson assembly, Dirichlet, 200 PCG")
    raise SystemExit(f"unknown workload {name}")


def host_cpu():
    """CPU model and logical core count of this host."""
    model = ""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(sample_n: int, workload: str = "hex128"):
    """The oracle, as is, on the same recipe at sample_n^3 (bounded CPU time):
    the serial parity build on one thread, then the all-core timing build
    (elements in colour order, PCG kernels over rows) on every thread it gets
    (OMP_NUM_THREADS, else every core).  value = the all-core rate."""
    import meshgen
    import oracle
    from oracle import omp
    recipe = {"hex128": (meshgen.cfg1, "hex08-"), "hex64": (meshgen.cfg1, "hex08-"),
              "tet128": (meshgen.cfg2, "tet04-6x"), "hybrid128": (meshgen.hybrid, "hybrid-")}
    make, label = recipe[workload]
    case = make(sample_n)
    ty = case.types
    pat = oracle.pattern(case.conn, case.n_nodes, ty)

    def run(mod, **kw):
        t0 = time.perf_counter()
        rp, ci, V, B = mod.assemble(case.coords, case.conn, oracle.OP_MOMENTUM, case.dt, case.u, case.rho, case.mu,
                                    pattern_=pat, types=ty, **kw)
        t1 = time.perf_counter()
        rp, ci, L, f = mod.assemble(case.coords, case.conn, oracle.OP_POISSON, case.dt, case.u, case.rho, None,
                                    pattern_=pat, types=ty, **kw)
        L, f = L[0], f[0]
        mod.dirichlet(rp, ci, L, f, case.dirichlet)
        t2 = time.perf_counter()
        mod.pcg(rp, ci, L, f, rtol=0.0, max_iter=CG_ITERS)
        t3 = time.perf_counter()
        return {"melem_s": case.n_elems / (t3 - t0) / 1e6, "assembly_melem_s": case.n_elems / (t1 - t0) / 1e6,
                "seconds": {"momentum": t1 - t0, "poisson_dirichlet": t2 - t1, "pcg": t3 - t2, "total": t3 - t0}}

    serial = run(oracle)
    colouring = omp.colour(case.conn, case.n_nodes, ty)     # set-up, like the GPU's upload: not timed
    threads = omp.threads()
    allc = run(omp, colouring=colouring)
    model, nproc = host_cpu()
    return {
        "value": allc["melem_s"], "unit": "Melem/s", "cores": threads, "kind": "oracle",
        "sample": (f"{label}{sample_n}^3 same recipe ({case.n_elems} elements): momentum+Poisson assembly, "
                   f"Dirichlet, {CG_ITERS} PCG; the C oracle on {threads} threads (colour-ordered element loop, "
                   f"{colouring[0]} colours) {allc['seconds']['total']:.1f} s, serial on 1 thread "
                   f"{serial['seconds']['total']:.1f} s"),
        "host_cpu": model, "nproc": nproc, "threads": threads,
        "all_threads": allc, "one_thread": serial,
        "assembly_melem_s": allc["assembly_melem_s"],
    }


def serve_measure(nreq, slots, threads, budget_gb, modes=("saturated", "load0.8", "load1.5"), records=None):
    """Serving workload: the first nreq requests of the serving stream,
    independent HEX08 cubes (side 8..96, log-uniform), each a momentum +
    Poisson assembly and a Jacobi-PCG solve to a true relative residual of
    1e-8.  Sequential FP64 (FIFO, one request at a time through the plain API)
    against the batching server: everything queued at once ("saturated") and
    Poisson arrivals at 0.8x / 1.5x the measured sequential capacity."""
    import concurrent.futures as cf
    import threading
    import torch
    import meshgen
    import paper_2107_11541_amd as fe

    t_unit, sides = meshgen.serving_stream(nreq, qps=1.0)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        cases = list(ex.map(lambda a: meshgen.serving_case(a[0], int(a[1])), enumerate(sides)))
    elems = np.array([c.n_elems for c in cases])
    log(f"serving: generated {nreq} requests (sides {sides.min()}..{sides.max()}, {int(elems.sum())} elements) "
        f"in {time.perf_counter() - t0:.1f} s")
    ctx = fe.Context(0)
    RTOL = 1e-8

    def run_plain(c):
        # a mesh assembled and solved once: the coloured blocks (no owner plan
        # to build) and the general SpMV (no symmetric map to build), as served
        mesh = fe.Mesh(ctx, c.elem_type, c.coords, c.conn, c.dirichlet, renumber=True, coloured=True,
                       symmetric_spmv=False)
        u = mesh.to_mesh(torch.as_tensor(c.u, device="cuda"))
        rho = mesh.to_mesh(torch.as_tensor(c.rho, device="cuda"))
        mu = mesh.to_mesh(torch.as_tensor(c.mu, device="cuda"))
        fe.assemble(mesh, fe.MOMENTUM, c.dt, u, rho, mu)
        L, f, _ = fe.assemble(mesh, fe.POISSON, c.dt, u, rho)
        fe.apply_dirichlet(mesh, L, f)
        x, info = fe.cg_solve(mesh, L[0], f[0], rtol=RTOL, max_iter=20000)
        xu = mesh.to_user(x).cpu().numpy()
        mesh.close()
        return xu, info

    # warm-up (library, kernels, allocator)
    run_plain(meshgen.serving_case(10**6, 12))
    torch.cuda.synchronize()
    seq_s = np.zeros(nreq)
    seq_res = np.zeros(nreq)
    t_all = time.perf_counter()
    for i, c in enumerate(cases):
        t0 = time.perf_counter()
        _, info = run_plain(c)
        seq_s[i] = time.perf_counter() - t0
        seq_res[i] = info["true_rel_residual"]
        if records is not None:
            records.append({"record": "request", "mode": "sequential_fp64", "request": i, "side": int(sides[i]),
                            "elements": int(elems[i]), "service_ms": seq_s[i] * 1e3,
                            "iterations": info["iterations"], "true_rel_residual": info["true_rel_residual"]})
    seq_total = time.perf_counter() - t_all
    mean_s = float(seq_s.mean())
    log(f"sequential FP64: {nreq / seq_total:.2f} solves/s, mean service {mean_s * 1e3:.1f} ms, "
        f"max true residual {seq_res.max():.2e}")

    def fifo_latency(arr):
        done, out = 0.0, np.zeros(nreq)
        for i in range(nreq):
            done = max(arr[i], done) + seq_s[i]
            out[i] = done - arr[i]
        return out

    def run_served(qps, mode):
        srv = fe.Server(ctx, hbm_budget=budget_gb << 30, max_slots=slots, host_threads=threads)
        arr = t_unit / qps if qps else np.zeros(nreq)
        tickets = [None] * nreq

        def feeder():
            t0 = time.perf_counter()
            for i, c in enumerate(cases):
                dt = arr[i] - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
                tickets[i] = srv.submit(c.elem_type, c.coords, c.conn, c.dirichlet, c.dt, c.u, c.rho, c.mu,
                                        rtol=RTOL, max_iter=20000)

        t0 = time.perf_counter()
        th = threading.Thread(target=feeder)
        th.start()
        res = []
        for i in range(nreq):
            while tickets[i] is None:
                time.sleep(0.0005)
            res.append(srv.wait(tickets[i]))
        th.join()
        wall = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        lat = np.array([r["total_ms"] for r in res])
        bad = [r for r in res if r["status"] != 0 or not r["true_rel_residual"] <= RTOL * 1.0001]
        if records is not None:
            for i, r in enumerate(res):
                records.append({"record": "request", "mode": mode, "request": i, "side": int(sides[i]),
                                "elements": int(elems[i]), "arrival_s": float(arr[i]), "status": r["status"],
                                **{k: r[k] for k in ("plan_ms", "wait_ms", "run_ms", "total_ms", "iterations",
                                                     "true_rel_residual")}})
        return {"qps_offered": qps, "solves_per_s": nreq / wall, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "mean_batch": st["mean_batch"],
                "max_true_rel_residual": float(max(r["true_rel_residual"] for r in res)), "failed": len(bad),
                "plan_ms_mean": float(np.mean([r["plan_ms"] for r in res])),
                "wait_ms_mean": float(np.mean([r["wait_ms"] for r in res])),
                "run_ms_mean": float(np.mean([r["run_ms"] for r in res]))}

    cap = 1.0 / mean_s
    loads = {"load0.8": 0.8, "load1.5": 1.5}
    runs = {}
    for name in modes:
        runs[name] = run_served(None if name == "saturated" else loads[name] * cap, name)
        log(f"served {name}: {json.dumps(runs[name])}")
    seq = {"solves_per_s": nreq / seq_total, "mean_service_ms": mean_s * 1e3,
           "max_true_rel_residual": float(seq_res.max())}
    for name in modes:
        if name in loads:
            lat = fifo_latency(t_unit / (loads[name] * cap))
            seq[f"p50_ms_at_{name}"] = float(np.percentile(lat, 50)) * 1e3
            seq[f"p99_ms_at_{name}"] = float(np.percentile(lat, 99)) * 1e3
    ctx.close()
    return {"workload": (f"serve-hex08-cubes-8..96-log-uniform, first {nreq} requests of the stream, "
                         f"momentum+Poisson assembly + PCG to true rel residual 1e-8"),
            "requests": nreq, "elements_total": int(elems.sum()), "slots": slots, "planner_threads": threads,
            "arena_gb": budget_gb, "sequential_fp64": seq, "served": runs,
            "speedup_saturated_vs_sequential": (runs["saturated"]["solves_per_s"] / seq["solves_per_s"]
                                                if "saturated" in runs else None)}


def write_records(path, line, records):
    """JSONL: one record per request of the serving runs, then the run's line."""
    if not path:
        return
    with open(path, "a") as fh:
        for r in records:
            fh.write(json.dumps(r) + "\n")
        fh.write(json.dumps(dict(line, record="run", time=time.time())) + "\n")


def serve_bench(args):
    records = [] if args.records else None
    r = serve_measure(args.serve_requests, args.serve_slots, args.serve_threads, args.serve_budget_gb,
                      records=records)
    line = {
        "metric": "served solves/s and p99 at 1e-8 rel err",
        "value": r["served"]["saturated"]["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {k: r[k] for k in ("workload", "requests", "elements_total", "slots", "planner_threads",
                                      "arena_gb")},
        "sequential_fp64": r["sequential_fp64"], "served": r["served"],
    }
    write_records(args.records, line, records or [])
    print(json.dumps(line), flush=True)


def cfg4_measure(n, reps):
    """256^3 HEX08 (jitter 15 %, 5 species): the momentum matrix with its 3
    right-hand sides, 5 scalar-transport matrices with theirs and the Poisson
    system, then the Poisson solve to a true relative residual of 1e-8 twice:
    FP64 Jacobi-PCG, and FP32 Jacobi-PCG inside FP64 iterative refinement;
    each solution's relative error against the other is reported."""
    import torch
    import meshgen
    import paper_2107_11541_amd as fe

    t0 = time.perf_counter()
    case = meshgen.cfg4(n)
    log(f"cfg4 {n}^3: N={case.n_nodes} E={case.n_elems} generated in {time.perf_counter() - t0:.1f} s")
    ctx = fe.Context(0)
    t0 = time.perf_counter()
    mesh = fe.Mesh(ctx, case.nen, case.coords, case.conn, case.dirichlet, renumber=True)
    upload_s = time.perf_counter() - t0
    dev = "cuda"
    u = mesh.to_mesh(torch.as_tensor(case.u, device=dev))
    rho = mesh.to_mesh(torch.as_tensor(case.rho, device=dev))
    mu = mesh.to_mesh(torch.as_tensor(case.mu, device=dev))
    Y = mesh.to_mesh(torch.as_tensor(case.Y, device=dev))
    N, nnz, E = mesh.n_nodes, mesh.nnz, mesh.n_elems
    Vm = torch.empty((1, nnz), dtype=torch.float64, device=dev)
    Bm = torch.empty((3, N), dtype=torch.float64, device=dev)
    Vs = torch.empty((5, nnz), dtype=torch.float64, device=dev)
    Bs = torch.empty((5, N), dtype=torch.float64, device=dev)
    L = torch.empty((1, nnz), dtype=torch.float64, device=dev)
    f = torch.empty((1, N), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    log(f"cfg4 uploaded in {upload_s:.1f} s, nnz={nnz}, device memory {torch.cuda.memory_allocated() / 2**30:.1f} GiB")

    def timed(fn):
        fn()
        ctx.profile(True)
        for _ in range(reps):
            fn()
        k, ms = ctx.profile_read(1)
        ctx.profile(False)
        return ms / k
    ms = {
        "momentum": timed(lambda: fe.assemble(mesh, fe.MOMENTUM, case.dt, u, rho, mu, values=Vm, rhs=Bm)),
        "scalars5": timed(lambda: fe.assemble(mesh, fe.SCALAR, case.dt, u, rho, Y=Y, D=case.D, values=Vs,
                                              rhs=Bs)) / 5,
        "poisson": timed(lambda: fe.assemble(mesh, fe.POISSON, case.dt, u, rho, values=L, rhs=f)),
    }
    del Vs, Bs
    total_ms = ms["momentum"] + 5 * ms["scalars5"] + ms["poisson"]
    fe.apply_dirichlet(mesh, L, f)
    torch.cuda.synchronize()
    solves, xs = {}, {}
    for name, prec in (("fp64_pcg", fe.FP64), ("mixed_ir", fe.MIXED)):
        # untimed warm-up: the first solve of a precision allocates its work
        # vectors (and, mixed, the FP32 value copy), builds the symmetric
        # SpMV's map (first solve on the mesh) and records its iteration
        # graph; a time-stepping code pays that once
        x = torch.zeros(N, dtype=torch.float64, device=dev)
        fe.cg_solve(mesh, L[0], f[0], x=x, rtol=1e-8, max_iter=16, precision=prec, raise_on_noconv=False)
        x = torch.zeros(N, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = fe.cg_solve(mesh, L[0], f[0], x=x, rtol=1e-8, max_iter=20000, precision=prec)
        torch.cuda.synchronize()
        solves[name] = dict(info, seconds=time.perf_counter() - t0)
        xs[name] = x
        log(f"cfg4 {name}: {solves[name]}")
    # the two solutions against each other (both at true rel residual <= 1e-8)
    solves["mixed_vs_fp64_rel_solution_diff"] = float(torch.linalg.norm(xs["mixed_ir"] - xs["fp64_pcg"]) /
                                                      torch.linalg.norm(xs["fp64_pcg"]))
    out = {
        "workload": (f"hex08-{n}^3-jitter15-5species: 1 momentum + 5 scalar + 1 Poisson matrix, "
                     f"Poisson solve to true rel residual 1e-8"),
        "elements": E, "nodes": N, "nnz": nnz,
        "assembly_melem_s_8_equations": E / (total_ms * 1e-3) / 1e6,
        "assembly_ms": dict(ms, all_8_equations=total_ms),
        "assembly_melem_s": {k: E / (v * 1e-3) / 1e6 for k, v in ms.items()},
        "solve": solves,
        "ir_speedup": solves["fp64_pcg"]["seconds"] / solves["mixed_ir"]["seconds"],
        "upload_s": upload_s,
    }
    mesh.close()
    ctx.close()
    return out


def cfg4_bench(args):
    r = cfg4_measure(args.cfg4_n, args.steps)
    line = {
        "metric": "Melem/s assembled (8 equations) and Poisson solve time to 1e-8: FP64 PCG vs FP32-in-FP64 IR",
        "value": r["assembly_melem_s_8_equations"], "unit": "Melem/s", "n_gpus": 1, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {k: r[k] for k in ("workload", "elements", "nodes", "nnz")},
        **{k: r[k] for k in ("assembly_ms", "assembly_melem_s", "solve", "ir_speedup", "upload_s")},
    }
    write_records(args.records, line, [])
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="hex128")
    ap.add_argument("--cpu-sample-n", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cfg4-n", type=int, default=256)
    ap.add_argument("--serve-requests", type=int, default=400)
    ap.add_argument("--no-serving", action="store_true", help="default workload: skip the serving sub-run")
    ap.add_argument("--no-cfg4", action="store_true", help="default workload: skip the 256^3 sub-run")
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--serve-threads", type=int, default=12)
    ap.add_argument("--serve-budget-gb", type=int, default=32)
    ap.add_argument("--records", default=None,
                    help="append JSONL records (one per served request, one per run) to this file")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 512 MiB device copy 3 times (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU (the multi-GPU domain decomposition is designed, "
              "not implemented); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2107_11541_amd as fe

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if args.copy_probe:
        a = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")   # 512 MiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel() * 8, "copies": 3}))
        return
    if args.workload == "serve":
        serve_bench(args)
        return
    if args.workload == "cfg4":
        cfg4_bench(args)
        return
    case, wl = make_workload(args.workload)
    log(f"workload {wl}: N={case.n_nodes} E={case.n_elems}")
    ctx = fe.Context(0)
    t0 = time.perf_counter()
    if case.types is None:
        mesh = fe.Mesh(ctx, case.nen, case.coords, case.conn, case.dirichlet, renumber=True)
        conn_entries = case.n_elems * case.nen
        type_counts = {str(case.nen): case.n_elems}
    else:
        mesh = fe.Mesh(ctx, fe.HYBRID, case.coords, case.conn, case.dirichlet, renumber=True, types=case.types)
        conn_entries = int(case.types.astype(np.int64).sum())
        type_counts = {str(t): int(c) for t, c in enumerate(np.bincount(case.types)) if c}
    upload_s = time.perf_counter() - t0
    info = mesh.info()
    log(f"mesh uploaded in {upload_s:.2f} s: nnz={mesh.nnz} blocks={info['n_blocks']} colours={info['n_colors']}")
    dev = "cuda"
    u = mesh.to_mesh(torch.as_tensor(case.u, device=dev))
    rho = mesh.to_mesh(torch.as_tensor(case.rho, device=dev))
    mu = mesh.to_mesh(torch.as_tensor(case.mu, device=dev))
    N, nnz, E = mesh.n_nodes, mesh.nnz, mesh.n_elems
    Vm = torch.empty((1, nnz), dtype=torch.float64, device=dev)
    Bm = torch.empty((3, N), dtype=torch.float64, device=dev)
    L = torch.empty((1, nnz), dtype=torch.float64, device=dev)
    f = torch.empty((1, N), dtype=torch.float64, device=dev)
    x = torch.zeros(N, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    last = {}

    def step():
        fe.assemble(mesh, fe.MOMENTUM, case.dt, u, rho, mu, values=Vm, rhs=Bm)
        fe.assemble(mesh, fe.POISSON, case.dt, u, rho, values=L, rhs=f)
        fe.apply_dirichlet(mesh, L, f)
        x.zero_()
        _, cg = fe.cg_solve(mesh, L, f, x=x, rtol=0.0, max_iter=CG_ITERS)
        last["cg"] = cg

    for i in range(args.warmup):
        step()
        log(f"warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step")
    # Per-kernel times come from separate steps with the library's event
    # brackets on (which launch every PCG kernel on its own instead of
    # replaying recorded iterations); they are not part of the timed region.
    prof_steps = max(1, min(args.steps, 3))
    ctx.profile(True)
    for i in range(prof_steps):
        step()
    torch.cuda.synchronize()
    n_spmv, ms_spmv = ctx.profile_read(0)
    n_asm, ms_asm = ctx.profile_read(1)
    n_upd, ms_upd = ctx.profile_read(2)
    n_dir, ms_dir = ctx.profile_read(3)
    ctx.profile(False)

    # per-operator assembly times (outside the timed region)
    def time_op(fn, reps=5):
        ctx.profile(True)
        for _ in range(reps):
            fn()
        n, ms = ctx.profile_read(1)
        ctx.profile(False)
        return ms / n
    ms_mom = time_op(lambda: fe.assemble(mesh, fe.MOMENTUM, case.dt, u, rho, mu, values=Vm, rhs=Bm))
    ms_poi = time_op(lambda: fe.assemble(mesh, fe.POISSON, case.dt, u, rho, values=L, rhs=f))
    # mixed-precision momentum assembly (FP32 quadrature, FP64 geometry and
    # accumulation): its rate and its error against the FP64 assembly
    Vx = torch.empty_like(Vm)
    Bx = torch.empty_like(Bm)
    ms_mix = time_op(lambda: fe.assemble(mesh, fe.MOMENTUM, case.dt, u, rho, mu, precision=fe.MIXED, values=Vx,
                                         rhs=Bx))
    fe.assemble(mesh, fe.MOMENTUM, case.dt, u, rho, mu, values=Vm, rhs=Bm)
    torch.cuda.synchronize()
    mixed_err = {"values_rel_frobenius": float(torch.linalg.norm(Vx - Vm) / torch.linalg.norm(Vm)),
                 "rhs_rel": float(torch.linalg.norm(Bx - Bm) / torch.linalg.norm(Bm))}
    del Vx, Bx

    # explicit step (Algorithm 1's Runge-Kutta stages, pressure solve and
    # correction), outside the timed region: one element-vector residual pass
    # and one whole fractional step to a pressure residual of 1e-8
    R4 = torch.empty((4, N), dtype=torch.float64, device=dev)
    ctx.profile(True)
    for _ in range(5):
        fe.residual(mesh, u, rho, mu, out=R4)
    n_res, ms_res = ctx.profile_read(4)
    ctx.profile(False)
    ctx.profile(True)
    for _ in range(5):
        fe.residual(mesh, u, rho, mu, out=R4, form=fe.FULL_STRESS | fe.EMAC)
    n_rfe, ms_rfe = ctx.profile_read(4)
    ctx.profile(False)
    del R4
    # scalar transport (heat, species): residual pass and one explicit step,
    # the first velocity component standing in for the scalar
    Ysc = u[0].clone()
    S2 = torch.empty((2, N), dtype=torch.float64, device=dev)
    ctx.profile(True)
    for _ in range(5):
        fe.scalar_residual(mesh, u, rho, Ysc, 1e-5, out=S2)
    n_sr, ms_sr = ctx.profile_read(4)
    ctx.profile(False)
    fe.scalar_step(mesh, case.dt, u, rho, 1e-5, Ysc)     # allocates its buffer
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fe.scalar_step(mesh, case.dt, u, rho, 1e-5, Ysc)
    torch.cuda.synchronize()
    scalar = {"scalar_residual_ms": ms_sr / n_sr, "scalar_step_ms": (time.perf_counter() - t0) * 1e3}
    del Ysc, S2
    wall = {}
    if case.wall_nen is not None:
        # boundary assembly: the wall model on the z = 0 faces, exchange
        # distance one cell; the fractional step below includes it
        mesh.set_wall(case.wall_nen, case.wall_conn, 1.0 / case.n)
        T3 = torch.empty((3, N), dtype=torch.float64, device=dev)
        ctx.profile(True)
        for _ in range(5):
            fe.wall_traction(mesh, u, rho, mu, out=T3)
        n_w, ms_w = ctx.profile_read(4)
        ctx.profile(False)
        del T3
        wall = {"wall_faces": int(case.wall_nen.shape[0]), "wall_traction_ms": ms_w / n_w}
    fe.assemble(mesh, fe.POISSON, case.dt, u, rho, values=L, rhs=f)
    fe.apply_dirichlet(mesh, L, f)
    us = u.clone()
    ps = torch.zeros(N, dtype=torch.float64, device=dev)
    fe.fractional_step(mesh, case.dt, rho, mu, L[0], us, ps, rtol=1e-8)   # allocates the step buffers
    us.copy_(u)
    ps.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_info = fe.fractional_step(mesh, case.dt, rho, mu, L[0], us, ps, rtol=1e-8)
    torch.cuda.synchronize()
    step_ms = (time.perf_counter() - t0) * 1e3
    # the same step with the pressure solved in mixed precision
    us.copy_(u)
    ps.zero_()
    fe.fractional_step(mesh, case.dt, rho, mu, L[0], us, ps, rtol=1e-8, precision=fe.MIXED)   # FP32 buffers
    us.copy_(u)
    ps.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_mixed = fe.fractional_step(mesh, case.dt, rho, mu, L[0], us, ps, rtol=1e-8, precision=fe.MIXED)
    torch.cuda.synchronize()
    step_mixed_ms = (time.perf_counter() - t0) * 1e3
    del us, ps
    explicit = {"residual_pass_ms": ms_res / n_res, "residual_melem_s": E / (ms_res / n_res * 1e-3) / 1e6,
                "fractional_step_mixed_pressure_ms": step_mixed_ms,
                "mixed_pressure_true_rel_residual": step_mixed["cg_true_rel_residual"],
                "residual_full_stress_emac_ms": ms_rfe / n_rfe,
                "fractional_step_ms": step_ms, "pressure_cg_iterations": step_info["cg_iterations"],
                "pressure_true_rel_residual": step_info["cg_true_rel_residual"], **wall, **scalar}
    log(f"explicit step: {json.dumps(explicit)}")

    spmv_us = ms_spmv / n_spmv * 1e3
    sb = spmv_bytes(nnz, N)
    achieved = sb / (spmv_us * 1e-6) / 1e9
    cg = last["cg"]
    line = {
        "metric": "Melem/s assembled + % HBM roofline; served solves/s and p99 at 1e-8 rel err",
        "value": E / (ms_step * 1e-3) / 1e6,
        "unit": "Melem/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl, "elements": E, "nodes": N, "nnz": nnz, "cg_iterations": CG_ITERS,
                   "blocks": info["n_blocks"], "colours": info["n_colors"],
                   "elements_by_nodes_per_element": type_counts},
        "roofline": roofline_entry(args.workload, sb, spmv_us, n_spmv, last["cg"]["symmetric_spmv"]),
        "breakdown": {
            "assembly_ms_per_step": ms_asm / prof_steps,
            "momentum_assembly_ms": ms_mom, "poisson_assembly_ms": ms_poi,
            "momentum_melem_s": E / (ms_mom * 1e-3) / 1e6, "poisson_melem_s": E / (ms_poi * 1e-3) / 1e6,
            "momentum_effective_gbs": momentum_bytes(nnz, N, conn_entries) / (ms_mom * 1e-3) / 1e9,
            "poisson_effective_gbs": poisson_bytes(nnz, N, conn_entries) / (ms_poi * 1e-3) / 1e9,
            "momentum_mixed_assembly_ms": ms_mix, "momentum_mixed_melem_s": E / (ms_mix * 1e-3) / 1e6,
            "momentum_mixed_vs_fp64": mixed_err,
            "assembly_roofline": assembly_roofline(args.workload, E, ms_mom, ms_poi, ms_mix),
            "dirichlet_ms": ms_dir / max(n_dir, 1),
            "cg_symmetric_spmv": cg["symmetric_spmv"],
            "cg_spmv_us": spmv_us, "cg_update_us": ms_upd / max(n_upd, 1) * 1e3,
            "cg_iteration_effective_gbs": (sb + 88 * N) / ((spmv_us + ms_upd / max(n_upd, 1) * 1e3) * 1e-6) / 1e9,
            "cg_rel_residual_after_200": cg["rel_residual"], "cg_true_rel_residual": cg["true_rel_residual"],
            "upload_s": upload_s,
            "explicit_step": explicit,
        },
    }
    counted = measured_valu(args.workload)
    if counted and "residual_fp64_flops_per_element" in counted:
        tf = counted["residual_fp64_flops_per_element"] * E / (explicit["residual_pass_ms"] * 1e-3) / 1e12
        explicit["residual_fp64_tflops"] = tf
        explicit["residual_fp64_frac"] = tf / FP64_PEAK_TFLOPS
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle on the same recipe")
        n_cpu = args.cpu_sample_n if args.workload in ("hex128", "hex64") else min(args.cpu_sample_n, 64)
        line["cpu_baseline"] = cpu_baseline(n_cpu, args.workload)
        log(f"cpu baseline: {json.dumps(line['cpu_baseline'])}")
    records = [] if args.records else None
    if args.workload == "hex128":
        # the metric's second half and the large single mesh, measured in the
        # same run (outside the timed region of the step above)
        del Vm, Bm, L, f, x, u, rho, mu
        mesh.close()
        ctx.close()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        if not args.no_serving:
            line["serving"] = serve_measure(args.serve_requests, args.serve_slots, args.serve_threads,
                                            args.serve_budget_gb, modes=("saturated", "load0.8"), records=records)
        if not args.no_cfg4:
            line["cfg4"] = cfg4_measure(args.cfg4_n, 5)
    write_records(args.records, line, records or [])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
