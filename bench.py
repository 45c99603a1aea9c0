#!/usr/bin/env python3
"""Benchmark of the deflated multi-shift, multi-RHS GMRES hot path on one GPU.

One step = one complete gdr_solve of the workload: GMRES-DR(60,20)-Sh on the
first right-hand side, the extra right-hand side v_{k+1}, the remaining
right-hand sides by batched GMRES(40)-Proj(20)-Sh with the correction, and
the FP64-refined cleanup, all shifts, to a true relative residual of 1e-8.
Inputs (links, right-hand sides) are synthetic and already resident in HBM
when the timed region starts.

value = seconds per all-shift solve (one right-hand side, every shift) in
mixed precision (FP32 matvec / Gram-Schmidt / basis, FP64 small problems,
accumulation and refinement). The same solve in plain FP64 is timed once for
the comparison, the dominant kernel class is timed with HIP events on the
library's stream for the roofline, and the CPU oracle is timed on a bounded
sample for the cpu_baseline.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload C4]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Dslash HBM GB/s; sec per all-shift solve at 1e-8, mixed+batched vs FP64"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def describe(name, cfg):
    lx, ly, lz, lt = cfg["dims"]
    kinds = sorted(set(k for k, _ in cfg["rhs"]))
    return ("%dx%dx%dx%d Wilson-Dirac (n=%d), %d %s RHS x %d shifts, GMRES-DR(%d,%d)-Sh + "
            "GMRES(%d)-Proj(%d)-Sh batched, tol %g" % (
                lx, ly, lz, lt, 12 * lx * ly * lz * lt, len(cfg["rhs"]), "/".join(kinds),
                len(cfg["sigmas"]), cfg["m_dr"], cfg["k"], cfg["m_proj"], cfg["k"], cfg["tol"]))


def cpu_baseline(cfg, links, kappa, b, sec_budget, gpu_steps):
    """Time the oracle's own GMRES-DR-Sh Arnoldi steps on this workload's
    first right-hand side (a bounded sample), fit t(j) = t_mv + (j+1) t_col
    and scale to the solve's observed Arnoldi steps per right-hand side."""
    import numpy as np
    from oracle import gmres, wilson
    op = wilson.WilsonOperator(links, kappa)
    m = cfg["m_dr"]
    n = op.n
    V = np.zeros((n, m + 1), dtype=np.complex128)
    H = np.zeros((m + 1, m), dtype=np.complex128)
    V[:, 0] = b / np.linalg.norm(b)
    times = []
    t_start = time.perf_counter()
    j = 0
    while j < m and (time.perf_counter() - t_start) < sec_budget:
        t0 = time.perf_counter()
        gmres.arnoldi_step(op, V, H, j)
        times.append(time.perf_counter() - t0)
        j += 1
    js = np.arange(len(times)) + 1.0
    if len(times) >= 2:
        t_col, t_mv = np.polyfit(js, np.array(times), 1)
        t_col = max(t_col, 0.0)
    else:
        t_mv, t_col = times[0], 0.0
    # observed step counts: (number of basis columns at each step) summed
    cost = sum(t_mv + (jj + 1) * t_col for jj in gpu_steps)
    threads = os.environ.get("OMP_NUM_THREADS") or str(len(os.sched_getaffinity(0)))
    return dict(cost=cost, t_mv=t_mv, t_col=t_col, steps=len(times),
                seconds=time.perf_counter() - t_start, threads=int(threads))


def host_info():
    """CPU model, logical CPUs visible to this process, and the BLAS/OpenMP
    thread settings the oracle runs with."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    env = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS",
                                          "MKL_NUM_THREADS") if os.environ.get(k)}
    blas = None
    try:
        import numpy as np
        cfg = np.show_config(mode="dicts")
        blas = cfg.get("Build Dependencies", {}).get("blas", {}).get("name")
    except Exception:
        pass
    return {"cpu_model": model, "nproc": len(os.sched_getaffinity(0)), "os_cpu_count": os.cpu_count(),
            "thread_env": env, "numpy_blas": blas}


def dslash_standalone(gdr, ops, vol, reps=100, nsets=3):
    """The Wilson operator alone: median per-launch time over `reps` launches
    rotating over `nsets` buffer sets (so the 256 MB Infinity Cache cannot hold
    one set), batch sizes 1, 3, 11, 12. Algorithmic bytes per launch count each
    link and spinor once (links amortised over the batch), the links as the
    operator stores them (gdr_op_link_bytes: 192 B/site for special unitary
    FP32 links kept as two rows, 288 for nine entries, 96 and 144 for FP16
    two-row and nine-entry storage, 576 FP64),
    spinors 192 B/site/vector FP32, 384 FP64. `gbs_480` restates FP32 rates
    on the nine-entry count (288 + 192 nb) for comparison with it."""
    import numpy as np
    rows = []
    for name, (op, prec) in ops.items():
        lk = float(gdr.gdr_op_link_bytes(op, prec))
        sp = 384.0 if prec == gdr.GDR_PREC_F64 else 192.0
        for nb in (1, 3, 11, 12):
            ms = gdr.gdr_op_dslash_bench(op, prec, nb, nsets, reps)
            med = float(np.median(ms))
            gbs = (lk + sp * nb) * vol / (med * 1e-3) / 1e9
            row = dict(variant=name, nvec=nb, us_median=med * 1e3, link_bytes_per_site=lk,
                       gbs=gbs, frac=gbs / HBM_PEAK_GBS)
            if prec != gdr.GDR_PREC_F64 and name == "f32":
                row["gbs_480"] = (288.0 + sp * nb) * vol / (med * 1e-3) / 1e9
            rows.append(row)
            log("bench: dslash %s nb=%d %.1f us %.0f GB/s (links %d B/site)"
                % (name, nb, med * 1e3, gbs, lk))
    return rows


TUNE_FORMS = {
    "dslash_r12": "0/1: vector-loop kernel, x-fastest / (z,t)-blocked tile order; "
                  "2/3: one block per tile and vector, same orders (one vector: 0/1 = orders)",
    "dslash_r12h": "as dslash_r12, for FP16 two-row links",
    "vrecombine_mfma": "strips per wavefront x quads per load group: 0 = 2x4, 1 = 4x2, 2 = 1x8",
    "blk_update": "blocks per member: 0 = default cap, 1 = 512, 2 = 1024 or 2048, 3 = 4096",
    "gs_update": "blocks per member: 0 = default cap, 1 = 512, 2 = 1024 or 2048, 3 = 4096",
    "vcombine": "blocks per member: 0 = 8192, 1 = 2048, 2 = 4096, 3 = 16384",
}


def tune_shapes(gdr):
    """The launch forms the tuner chose in this process, per kernel and shape."""
    out = {}
    for line in gdr.gdr_tune_report().splitlines():
        key, _, rest = line.partition(" -> ")
        if not rest:
            continue
        form, _, us = rest.partition(" (")
        out[key] = {"form": int(form), "us_per_unit": float(us.split()[0])}
    return {"chosen": out, "forms": TUNE_FORMS} if out else None


def counter_traffic(kernel_class, workload):
    """HBM bytes per launch of a kernel class from the committed rocprofv3
    counter summary (profiles/*_traffic.md), if it covers this class and
    workload and the kernel source is unchanged since the counters were taken;
    otherwise None."""
    import glob
    import hashlib
    for path in glob.glob(os.path.join(ROOT, "profiles", "*_traffic.md")):
        fields = {}
        for line in open(path):
            if ":" in line and not line.startswith(("|", "#", "`")):
                key, _, val = line.partition(":")
                fields[key.strip()] = val.strip()
        if fields.get("kernel_class") != kernel_class or fields.get("workload") != workload:
            continue
        src, _, digest = fields.get("source", "").partition(" sha256 ")
        try:
            data = open(os.path.join(ROOT, src), "rb").read()
        except OSError:
            return None
        if hashlib.sha256(data).hexdigest() != digest.strip():
            return None
        return float(fields["traffic_bytes_per_launch"])
    return None


def arnoldi_columns(st, cfg, nrhs):
    """Arnoldi steps of one solve as a list of basis widths j+1 (for the CPU
    extrapolation), from the library's counters."""
    m, k, mp = cfg["m_dr"], cfg["k"], cfg["m_proj"]
    steps = []
    c = st.s.cycles_dr
    if c > 0:
        steps += list(range(0, m))
        steps += list(range(k, m)) * (c - 1)
    nproj = st.s.cycles_extra + st.s.cycles_proj + st.s.cycles_cleanup
    steps += list(range(0, mp)) * nproj
    return steps


def operator_timings(a, gdr, synth, ctx, op, dims, kappa, links, n):
    """Standalone Wilson operator timings on the workload's lattice and, unless
    skipped, on the 32^3x64 lattice."""
    op16 = gdr.gdr_wilson_create(ctx, dims, (1, 1, 1, -1), kappa, links, gdr.GDR_LINKS_F16)
    dsl = dslash_standalone(gdr, {"f32": (op, gdr.GDR_PREC_F32),
                                  "f16link": (op16, gdr.GDR_PREC_F32),
                                  "f64": (op, gdr.GDR_PREC_F64)}, n // 12)
    gdr.gdr_op_destroy(op16)
    if a.workload != "C5" and not a.no_big_dslash:
        # the operator alone on the largest lattice (32^3x64, 25.2M unknowns):
        # its working set is far above the 256 MB Infinity Cache
        c5 = synth.CONFIGS["C5"]
        links5 = synth.gauge_links(c5["dims"], c5["eps"], c5["seed"])
        try:
            kappa5 = synth.kappa("C5")
        except KeyError:
            kappa5 = kappa   # the timing does not depend on the value
        ops5 = {}
        for name, storage in (("f32", gdr.GDR_LINKS_F32), ("f16link", gdr.GDR_LINKS_F16)):
            ops5[name] = gdr.gdr_wilson_create(ctx, c5["dims"], (1, 1, 1, -1), kappa5, links5,
                                               storage)
        del links5
        big = dslash_standalone(gdr, {"f32": (ops5["f32"], gdr.GDR_PREC_F32),
                                      "f16link": (ops5["f16link"], gdr.GDR_PREC_F32),
                                      "f64": (ops5["f32"], gdr.GDR_PREC_F64)},
                                ops5["f32"].n // 12)
        dsl = {"24x24x24x48": dsl, "32x32x32x64": big}
        for o in ops5.values():
            gdr.gdr_op_destroy(o)

    return dsl


def uneven_batch(a, gdr, synth, torch, np):
    """The uneven mixed batch: one 32^3x64 lattice with FP16-stored links
    (8 shifts, 4 Z4 RHS) solved concurrently with six 12^4 and four 16^4
    lattices (4 shifts, 2 RHS), each lattice on its own context and stream,
    Arnoldi cycles replayed from HIP graphs; the small lattices by one
    gdr_solve_many call with persistent work-list launches (--c5-persistent 1,
    the default) or each on a host thread of its own (0).
    value: wall time of the whole batch divided by its 24 right-hand sides;
    the same batch in plain FP64 (also concurrent, on contexts of its own) is
    timed first."""
    import threading
    inputs = []
    for name in synth.C5_GROUP:
        cfg = synth.CONFIGS[name]
        links = synth.gauge_links(cfg["dims"], cfg["eps"], cfg["seed"])
        B = np.stack([synth.make_rhs(cfg, kd, sd).ravel() for kd, sd in cfg["rhs"]])
        inputs.append((name, cfg, links, B))
        log("bench: inputs", name, cfg["dims"])

    def cu_stream(small):
        # a stream whose kernels run on part of the CUs: the small lattices on
        # a.c5_cu_split CUs of each XCD, the 32^3x64 lattice on the rest. The
        # set {32x + 8c + x} holds a.c5_cu_split CUs of every XCD whether mask
        # bit i names a CU of XCD i % 8 or of XCD i // 32.
        import ctypes
        ncu = torch.cuda.get_device_properties(0).multi_processor_count
        if ncu != 256:
            raise SystemExit("--c5-cu-split assumes 256 CUs in 8 XCDs (found %d CUs)" % ncu)
        sel = {32 * x + 8 * c + x for x in range(8) for c in range(a.c5_cu_split)}
        bits = [(i in sel) == small for i in range(256)]
        words = [sum(1 << b for b in range(32) if bits[32 * w + b]) for w in range(8)]
        hip = ctypes.CDLL("libamdhip64.so")
        h = ctypes.c_void_p()
        arr = (ctypes.c_uint32 * 8)(*words)
        rc = hip.hipExtStreamCreateWithCUMask(ctypes.byref(h), ctypes.c_uint32(8), arr)
        if rc != 0:
            raise SystemExit("hipExtStreamCreateWithCUMask failed: %d" % rc)
        return torch.cuda.ExternalStream(h.value)

    def make_runs():
        # one context, stream and operator per lattice; each context keeps
        # its own device-memory cache, so the FP64 and the mixed batch get
        # fresh contexts (the FP64 batch's cached buffers would otherwise
        # crowd the mixed one into allocating inside its timed region)
        out = []
        for name, cfg, links, B in inputs:
            stream = cu_stream(name != "C5") if a.c5_cu_split else torch.cuda.Stream()
            ctx = gdr.gdr_ctx_create(0, stream.cuda_stream)
            lst = gdr.GDR_LINKS_F16 if cfg.get("links") == "f16" else gdr.GDR_LINKS_F32
            if a.c5_links == "f32":
                lst = gdr.GDR_LINKS_F32
            op = gdr.gdr_wilson_create(ctx, cfg["dims"], (1, 1, 1, -1), synth.kappa(name), links,
                                       lst)
            with torch.cuda.stream(stream):
                Bd = torch.from_numpy(B.ravel()).cuda()
                X = torch.zeros(len(cfg["rhs"]) * len(cfg["sigmas"]) * op.n,
                                dtype=torch.complex128, device="cuda")
            stream.synchronize()
            out.append(dict(name=name, cfg=cfg, op=op, ctx=ctx, stream=stream, Bd=Bd, X=X))
        return out

    def drop(rs):
        torch.cuda.synchronize()
        for r in rs:
            gdr.gdr_op_destroy(r["op"])
            gdr.gdr_ctx_destroy(r["ctx"])
        rs.clear()
        torch.cuda.empty_cache()

    def batch(prec, profile_big=False):
        if prec == gdr.GDR_PREC_MIXED and a.c5_persistent:
            return batch_persistent(profile_big)

        def solve(r):
            cfg = r["cfg"]
            p = gdr.gdr_params_default(m_dr=cfg["m_dr"], k=cfg["k"], m_proj=cfg["m_proj"],
                                       tol=cfg["tol"], tol_extra=cfg["tol_extra"], precision=prec,
                                       use_graph=1, refine_floor=a.refine_floor, m_clean=a.m_clean)
            if profile_big and r["name"] == "C5":
                # kernel classes of the critical path (the 32^3x64 lattice)
                # timed with HIP events on its stream; the small lattices keep
                # their graph replays (profiling runs a context's cycles eagerly)
                p.profile = 0xFF
            st = gdr.Stats(len(cfg["rhs"]), len(cfg["sigmas"]))
            t0 = time.perf_counter()
            r["rc"] = gdr.gdr_solve(r["op"], cfg["sigmas"], r["Bd"], r["X"], p, st)
            r["sec"] = time.perf_counter() - t0
            r["st"] = st
        threads = [threading.Thread(target=solve, args=(r,)) for r in runs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def batch_persistent(profile_big):
        # the 32^3x64 lattice by gdr_solve on its own thread; the ten small
        # lattices by one gdr_solve_many call (params.persistent = 1: their
        # first right-hand sides as one batch of work-list launches, then each
        # lattice's later right-hand side and cleanup on its own context)
        big = next(r for r in runs if r["name"] == "C5")
        small = [r for r in runs if r["name"] != "C5"]
        c0 = small[0]["cfg"]

        def solve_big():
            cfg = big["cfg"]
            p = gdr.gdr_params_default(m_dr=cfg["m_dr"], k=cfg["k"], m_proj=cfg["m_proj"],
                                       tol=cfg["tol"], tol_extra=cfg["tol_extra"],
                                       precision=gdr.GDR_PREC_MIXED, use_graph=1,
                                       refine_floor=a.refine_floor, m_clean=a.m_clean)
            if profile_big:
                p.profile = 0xFF
            st = gdr.Stats(len(cfg["rhs"]), len(cfg["sigmas"]))
            t0 = time.perf_counter()
            big["rc"] = gdr.gdr_solve(big["op"], cfg["sigmas"], big["Bd"], big["X"], p, st)
            big["sec"] = time.perf_counter() - t0
            big["st"] = st

        def solve_small():
            p = gdr.gdr_params_default(m_dr=c0["m_dr"], k=c0["k"], m_proj=c0["m_proj"],
                                       tol=c0["tol"], tol_extra=c0["tol_extra"],
                                       precision=gdr.GDR_PREC_MIXED, use_graph=1,
                                       refine_floor=a.refine_floor, m_clean=a.m_clean,
                                       persistent=1)
            sts = [gdr.Stats(len(r["cfg"]["rhs"]), len(r["cfg"]["sigmas"])) for r in small]
            rc = gdr.gdr_solve_many([r["op"] for r in small], c0["sigmas"],
                                    [r["Bd"] for r in small], [r["X"] for r in small], p, sts)
            for r, st in zip(small, sts):
                r["rc"], r["st"], r["sec"] = rc, st, st.s.t_total

        threads = [threading.Thread(target=solve_big), threading.Thread(target=solve_small)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    nrhs = sum(len(cfg["rhs"]) for _, cfg, _, _ in inputs)
    fp64 = None
    runs = []
    if not a.no_fp64:
        runs += make_runs()
        for w in range(a.warmup):
            batch(gdr.GDR_PREC_F64)
        wall64 = batch(gdr.GDR_PREC_F64)
        fp64 = dict(sec_per_all_shift_solve=wall64 / nrhs, wall=wall64,
                    max_true_resid=max(float(r["st"].resid.max()) for r in runs),
                    rc=[r["rc"] for r in runs])
        log("bench: fp64 batch", fp64)
        drop(runs)
    runs += make_runs()
    for w in range(a.warmup):
        batch(gdr.GDR_PREC_MIXED)
    walls = []
    kern = {}
    for _ in range(a.steps):
        walls.append(batch(gdr.GDR_PREC_MIXED, profile_big=True))
        big = next(r for r in runs if r["name"] == "C5")
        for name, d in big["st"].kernels().items():
            e = kern.setdefault(name, dict(ms=0.0, bytes=0.0, flops=0.0, launches=0))
            for key in e:
                e[key] += d[key]
    wall = sum(walls) / len(walls)
    per = {r["name"]: dict(sec=r["sec"], rc=r["rc"], **{k: v for k, v in r["st"].as_dict().items()
                                                      if k.startswith(("mvp", "cycles", "t_phase"))},
                           max_true_resid=float(r["st"].resid.max())) for r in runs}
    if fp64 is not None:
        fp64["speedup_mixed_vs_fp64"] = fp64["wall"] / wall
    dom = max((k for k in kern if kern[k]["bytes"] > 0), key=lambda k: kern[k]["ms"])
    kd = kern[dom]
    achieved = kd["bytes"] / (kd["ms"] * 1e-3) / 1e9
    total_ms = sum(v["ms"] for v in kern.values())
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": counter_traffic(dom, "C5"),
                "algorithmic_bytes_per_launch": kd["bytes"] / kd["launches"] if kd["launches"] else None,
                "scope": "the 32x32x32x64 lattice's kernels (the critical path), timed with HIP events "
                         "on its stream while the ten small lattices run concurrently",
                "kernel_share_of_timed_kernel_ms": kd["ms"] / total_ms if total_ms else None}
    cpu = None
    if not a.no_cpu:
        # the oracle's Arnoldi steps on one lattice of each size (bounded
        # samples), each lattice's own Arnoldi step count from its solve
        cost = 0.0
        samples = []
        budget = {"C5": 0.6 * a.cpu_seconds, "C5a": 0.2 * a.cpu_seconds, "C5b": 0.2 * a.cpu_seconds}
        fits = {}
        for name, cfg, links, B in inputs:
            group = name if name == "C5" else name[:3]
            if group not in fits:
                c = cpu_baseline(cfg, links, synth.kappa(name), B[0], budget[group], [])
                fits[group] = c
                samples.append("%d steps on %s in %.1f s (t = %.3f s + (j+1) * %.4f s)"
                               % (c["steps"], "x".join(map(str, cfg["dims"])), c["seconds"],
                                  c["t_mv"], c["t_col"]))
            c = fits[group]
            r = next(x for x in runs if x["name"] == name)
            steps = arnoldi_columns(r["st"], cfg, len(cfg["rhs"]))
            cost += sum(c["t_mv"] + (j + 1) * c["t_col"] for j in steps)
        cpu = dict(value=cost / nrhs, unit="s", cores=fits["C5"]["threads"], kind="oracle",
                   host=host_info(),
                   sample="oracle GMRES-DR-Sh Arnoldi steps (matvec + CGS2): " + "; ".join(samples)
                          + "; scaled to each lattice's own Arnoldi steps in the GPU solve, summed, "
                            "per RHS (extrapolated; the oracle solves the lattices one after another)")
        log("bench: cpu", cpu)
    out = {
        "metric": METRIC, "value": wall / nrhs, "unit": "s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": wall * 1e3, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "uneven mixed batch, solved concurrently: 32x32x32x64 Wilson-Dirac "
                               "(n=25165824, FP16-stored links) 4 Z4 RHS x 8 shifts, GMRES-DR(60,20)-Sh + "
                               "GMRES(40)-Proj(20)-Sh; six 12^4 and four 16^4 lattices, 2 Z4 RHS x 4 "
                               "shifts, DR(40,15) + Proj(40,15); tol 1e-8; one context and stream per "
                               "lattice, Arnoldi cycles replayed from HIP graphs" +
                               ("; the ten small lattices in one gdr_solve_many call whose first "
                                "right-hand sides run as one batch of persistent work-list launches"
                                if a.c5_persistent else ""),
                   "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES"),
                   "name": "C5", "nrhs": nrhs, "global_batch": nrhs, "parallelism": "1 GPU",
                   "precision": "mixed: FP32 matvec/Gram-Schmidt/basis, FP64 small problems, "
                                "accumulation and refinement"},
        "roofline": roofline, "fp64": fp64, "cpu_baseline": cpu, "kernels_big_lattice": kern,
        "max_true_resid": max(v["max_true_resid"] for v in per.values()), "lattices": per,
        "step_walls_s": walls, "tune": tune_shapes(gdr),
    }
    print(json.dumps(out), flush=True)
    drop(runs)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps first (default 1; 2 for C5, whose first concurrent batch "
                         "after the FP64 one still grows the shared device-memory cache)")
    ap.add_argument("--workload", default="C4")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--cpu-e2e", action="store_true",
                    help="time the oracle's whole solve instead of a sample (small workloads)")
    ap.add_argument("--no-dslash", action="store_true")
    ap.add_argument("--no-big-dslash", action="store_true",
                    help="skip the standalone operator timing on the 32^3x64 lattice")
    ap.add_argument("--dslash-only", action="store_true",
                    help="only the standalone operator timings (no solves); prints their JSON")
    ap.add_argument("--sstep", type=int, default=None,
                    help="block size of the FP32 Arnoldi cycle (default: the library's)")
    ap.add_argument("--m-clean", type=int, default=0,
                    help="cycle length of the mixed-precision cleanup (0: library default)")
    ap.add_argument("--tol-extra", type=float, default=None,
                    help="tolerance of the extra right-hand side (default: the workload's)")
    ap.add_argument("--refine-floor", type=float, default=0.0,
                    help="inner tolerance floor of the cleanup's refinement rounds (0: library default)")
    ap.add_argument("--c5-links", choices=["f16", "f32"], default="f16",
                    help="link storage of the uneven batch's 32^3x64 lattice (default: the "
                         "workload's FP16)")
    ap.add_argument("--c5-cu-split", type=int, default=0,
                    help="uneven batch: the small lattices' streams on this many CUs of each XCD, "
                         "the 32^3x64 lattice's on the others (CU-masked streams; 0: all CUs)")
    ap.add_argument("--c5-persistent", type=int, choices=[0, 1], default=1,
                    help="uneven batch: the ten small lattices as one gdr_solve_many call with "
                         "persistent work-list launches (1) or on contexts of their own (0)")
    ap.add_argument("--hw-queues", type=int, default=12,
                    help="hardware queues per process for the uneven batch (C5; 0: the "
                         "environment's setting)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="end with a 256 MiB device copy (calibrates hardware byte counters)")
    a = ap.parse_args()
    if a.warmup is None:
        a.warmup = 2 if a.workload == "C5" else 1
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(requested --gpus %d)" % a.gpus, file=sys.stderr)
        sys.exit(2)

    if not 0 <= a.hw_queues <= 32:
        print("--hw-queues must be 0..32", file=sys.stderr)
        sys.exit(2)
    if a.workload == "C5" and a.hw_queues > 0:
        # eleven concurrent streams: more hardware queues than HIP's default 4
        # let the small lattices' launches stop queueing behind the large
        # one's (must be set before the HIP runtime starts)
        os.environ["GPU_MAX_HW_QUEUES"] = str(a.hw_queues)

    import numpy as np
    import torch

    import synth
    from paper_0707_0502_amd import gdr

    if a.workload == "C5":
        torch.cuda.init()
        uneven_batch(a, gdr, synth, torch, np)
        return
    cfg = synth.CONFIGS[a.workload]
    dims = cfg["dims"]
    log("bench: workload", a.workload, describe(a.workload, cfg))
    links = synth.gauge_links(dims, cfg["eps"], cfg["seed"])
    kappa = synth.kappa(a.workload)
    B = np.stack([synth.make_rhs(cfg, kd, s).ravel() for kd, s in cfg["rhs"]])
    sig = list(cfg["sigmas"])
    nrhs, ns = B.shape[0], len(sig)
    torch.cuda.init()
    ctx = gdr.gdr_ctx_create(0, torch.cuda.current_stream().cuda_stream)
    op = gdr.gdr_wilson_create(ctx, dims, (1, 1, 1, -1), kappa, links, gdr.GDR_LINKS_F32)
    n = op.n
    if a.dslash_only:
        print(json.dumps({"dslash_standalone": operator_timings(a, gdr, synth, ctx, op, dims, kappa,
                                                                links, n)}), flush=True)
        return
    Bd = torch.from_numpy(B.ravel()).cuda()
    X = torch.zeros(nrhs * ns * n, dtype=torch.complex128, device="cuda")
    del B

    def params(prec, profile):
        p = gdr.gdr_params_default(m_dr=cfg["m_dr"], k=cfg["k"], m_proj=cfg["m_proj"],
                                   tol=cfg["tol"],
                                   tol_extra=cfg["tol_extra"] if a.tol_extra is None else a.tol_extra,
                                   precision=prec, batch=1, profile=profile,
                                   m_clean=a.m_clean, refine_floor=a.refine_floor)
        if a.sstep is not None:
            p.sstep = a.sstep
        return p

    # the plain FP64 solve first, on a device no other solve has used yet
    fp64 = None
    if not a.no_fp64:
        st64 = gdr.Stats(nrhs, ns)
        X64 = torch.zeros_like(X)
        for w in range(a.warmup):   # the same warm-up as the mixed solve gets
            gdr.gdr_solve(op, sig, Bd, X64, params(gdr.GDR_PREC_F64, 0), gdr.Stats(nrhs, ns))
        torch.cuda.synchronize()
        tf0 = time.perf_counter()
        rc64 = gdr.gdr_solve(op, sig, Bd, X64, params(gdr.GDR_PREC_F64, 0), st64)
        torch.cuda.synchronize()
        tf = time.perf_counter() - tf0
        fp64 = dict(sec_per_all_shift_solve=tf / nrhs, rc=rc64,
                    max_true_resid=float(st64.resid.max()), counters=st64.as_dict())
        X64 = X64.cpu()   # compared with the mixed solution below

    pm = params(gdr.GDR_PREC_MIXED, 0xFF)
    for w in range(a.warmup):
        st = gdr.Stats(nrhs, ns)
        rc = gdr.gdr_solve(op, sig, Bd, X, pm, st)
        log("bench: warmup", w, "rc", rc, "t", round(st.s.t_total, 3), st.as_dict())
    torch.cuda.synchronize()
    kern = {}
    t0 = time.perf_counter()
    for s in range(a.steps):
        st = gdr.Stats(nrhs, ns)
        rc = gdr.gdr_solve(op, sig, Bd, X, pm, st)
        for name, d in st.kernels().items():
            e = kern.setdefault(name, dict(ms=0.0, bytes=0.0, flops=0.0, launches=0))
            for key in e:
                e[key] += d[key]
        log("bench: step", s, "rc", rc, "t", round(st.s.t_total, 3))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / a.steps
    value = ms_per_step / 1e3 / nrhs
    resid_max = float(st.resid.max())
    counters = st.as_dict()
    log("bench: mixed", counters, "max true resid %.3e" % resid_max)
    if fp64 is not None:
        Xm = X.cpu()
        fp64["speedup_mixed_vs_fp64"] = fp64["sec_per_all_shift_solve"] / value
        fp64["rel_diff_mixed_vs_fp64"] = float(torch.linalg.norm(X64 - Xm) / torch.linalg.norm(X64))
        del Xm, X64
        log("bench: fp64", fp64)

    # dominant kernel class by time, and the Wilson operator's own rate
    dom = max((k for k in kern if kern[k]["bytes"] > 0), key=lambda k: kern[k]["ms"])
    kd = kern[dom]
    achieved = kd["bytes"] / (kd["ms"] * 1e-3) / 1e9
    ds = kern["dslash"]
    dslash_gbs = ds["bytes"] / (ds["ms"] * 1e-3) / 1e9 if ds["ms"] > 0 else None
    total_ms = sum(v["ms"] for v in kern.values())

    dsl = None if a.no_dslash else operator_timings(a, gdr, synth, ctx, op, dims, kappa, links, n)

    cpu = None
    if not a.no_cpu and a.cpu_e2e:
        # the oracle's whole solve (every RHS and shift, the paper's order of
        # use) on the same inputs, timed end to end
        from oracle import gmres, wilson
        Bh = Bd.cpu().numpy().reshape(nrhs, n)
        t0c = time.perf_counter()
        ref = gmres.solve_all(wilson.WilsonOperator(links, kappa), Bh, sig, cfg["m_dr"], cfg["k"],
                              cfg["m_proj"], cfg["tol"], cfg["tol_extra"])
        tc = time.perf_counter() - t0c
        threads = os.environ.get("OMP_NUM_THREADS") or str(len(os.sched_getaffinity(0)))
        mv = sum(int(r.get("mvps", 0)) for r in ref["runs"])
        cpu = dict(value=tc / nrhs, unit="s", cores=int(threads), kind="oracle", host=host_info(),
                   sample="the oracle's complete FP64 solve of this workload (%d RHS x %d shifts, "
                          "%d products, max true residual %.1e) timed end to end: %.1f s"
                          % (nrhs, ns, mv, float(ref["resid"].max()), tc))
        log("bench: cpu", cpu)
    elif not a.no_cpu:
        b0 = Bd[:n].cpu().numpy()
        steps = arnoldi_columns(st, cfg, nrhs)
        c = cpu_baseline(cfg, links, kappa, b0, a.cpu_seconds, steps)
        cpu = dict(value=c["cost"] / nrhs, unit="s", cores=c["threads"], kind="oracle",
                   host=host_info(),
                   sample="%d oracle GMRES-DR-Sh Arnoldi steps (matvec + CGS2) on RHS 1 of the "
                          "same workload in %.1f s; fit t = %.3f s + (j+1) * %.4f s, scaled to the "
                          "%d Arnoldi steps the GPU solve took, per RHS (extrapolated)"
                          % (c["steps"], c["seconds"], c["t_mv"], c["t_col"], len(steps)))
        log("bench: cpu", cpu)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": describe(a.workload, cfg), "name": a.workload,
                   "precision": "mixed: FP32 matvec/Gram-Schmidt/basis, FP64 small problems, "
                                "accumulation and refinement",
                   "nrhs": nrhs, "shifts": ns, "global_batch": nrhs, "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": counter_traffic(dom, a.workload),
                     "algorithmic_bytes_per_launch": kd["bytes"] / kd["launches"] if kd["launches"] else None,
                     "kernel_share_of_timed_kernel_ms": kd["ms"] / total_ms if total_ms else None},
        "dslash": {"in_solver_gbs": dslash_gbs,
                   "in_solver_frac": (dslash_gbs / HBM_PEAK_GBS) if dslash_gbs else None,
                   "in_solver_launches": ds["launches"],
                   "standalone": dsl},
        "fp64": fp64,
        "cpu_baseline": cpu,
        "max_true_resid": resid_max,
        "counters": counters,
        "kernels": kern,
        "tune": tune_shapes(gdr),
    }
    print(json.dumps(out), flush=True)
    if a.copy_probe:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: copy probe 268435456 bytes read, 268435456 written")


if __name__ == "__main__":
    main()
