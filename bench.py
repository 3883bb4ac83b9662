"""Throughput of the lMBD hot path (energy + exact forces) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64|mixed]
                    [--workload plain|mixed] [--no-cpu-baseline] [--no-serve] [--serve-sweep]
                    [--no-mixed] [--no-two-point] [--no-two-radius]

A step is one complete evaluation (neighbour lists, local SCS at every
frequency, local MBD energies, all adjoints, forces) of the whole workload,
with inputs resident in device memory.  The default workload is 1,728 C atoms
in a periodic box at 2.0 g/cm^3 with a 6 A cutoff, 12 quadrature nodes and
n_max = 6, in FP64; the same workload is also timed in mixed precision, and
with the two-point Lorentzian SCS frequency model (SCS at omega = 0 and
omega_ref only) in both precisions, beside its deviation from the exact
frequency treatment, and in the two-radius regime (r_MBD,1 = 6 A, r_MBD,2 = 3 A,
K = B(9 A)) with sparse and with dense MBD products.  The
serving section replays 256 H/C/N/O requests (50-5,000 atoms) arriving as a
Poisson stream through the continuous-batching server in mixed precision,
and through a one-request-at-a-time FP64 server, and reports atoms/s with
p50/p99 latency.  Prints one JSON line.
"""
import argparse
import dataclasses
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "atoms/s lMBD energy+forces, FP64 plain vs mixed/served at <=1e-5 eV/atom; p99"
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def neighbour_counts(st, rc):
    """Atoms within rc of every atom, itself included (input analysis only)."""
    from scipy.spatial import cKDTree
    if st.cell is not None:
        # every periodic image within rc counts (a cube of edge L; rc may exceed L / 2)
        L = float(st.cell[0, 0])
        pts = np.mod(st.pos, L)
        m = int(np.ceil(rc / L))
        rng = np.arange(-m, m + 1)
        shifts = np.stack(np.meshgrid(rng, rng, rng, indexing="ij"), -1).reshape(-1, 3) * L
        tree = cKDTree((pts[None, :, :] + shifts[:, None, :]).reshape(-1, 3))
    else:
        tree = cKDTree(st.pos)
        pts = st.pos
    return np.array([len(x) for x in tree.query_ball_point(pts, rc - 1e-12)])


def scs_factor_flops(n1, nw):
    """Algorithmic FLOPs of the SCS factorisation: N^3/3 per (atom, frequency), N = 3 n1."""
    N = 3.0 * n1.astype(np.float64)
    return float(np.sum(nw * N ** 3 / 3.0))


def scs_solve_flops(n1, nw, n_tri):
    """Triangular solves with 3 right-hand sides: 3 N^2 per triangular solve and (atom, frequency)."""
    N = 3.0 * n1.astype(np.float64)
    return float(np.sum(nw * n_tri * 3.0 * N ** 2))


def source_digest(paths):
    """SHA-256 over kernel sources (ties a stored counter reading to the code it was taken on)."""
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


FACTOR_SOURCES = ["paper_2407_06409_amd/csrc/k_scs.hip", "paper_2407_06409_amd/csrc/lmbd_internal.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "scs_factor_C1728_fp64_traffic.md")


def stored_traffic():
    """HBM bytes per launch of the factorisation kernel from the committed counter
    summary, if it was taken on the current kernel sources (else None)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_digest") != source_digest(FACTOR_SOURCES):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def mbd_flops(nK, nq, n_max, forces):
    """Algorithmic FLOPs of the MBD stage: Krylov products (N3^2 x 3 n_q each) and,
    with forces, the Tbar product (N3^2 x 3 n_q n_max), of which only the lower
    triangle N3 (N3 + 1) / 2 is needed since Tbar is symmetric."""
    N3 = 3.0 * nK.astype(np.float64)
    ncol = 3 * nq
    prods = (n_max - 2) if forces else (math.ceil(n_max / 2) - 1)
    f = np.sum(prods * 2.0 * N3 ** 2 * ncol)
    if forces:
        f += np.sum(N3 * (N3 + 1.0) * ncol * n_max)
    return float(f)


_BASE = {}


def _baseline_worker_init():
    import torch
    torch.set_num_threads(1)


def _baseline_task(k):
    """One sampled central atom through the oracle as it stands; returns its timings."""
    import oracle
    from workloads import SPECIES_TABLE
    tm = {}
    w = np.zeros(_BASE["st"].n)
    w[k] = 1.0
    oracle.lmbd_energy_forces(_BASE["st"], _BASE["prm"], SPECIES_TABLE, weights=w, atoms=[k], timings=tm)
    return tm


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(st, cut, grid, n_sample=32):
    """The FP64 oracle on the host cores, on a bounded sample of the same workload.

    The sample is n_sample seeded central atoms of the box, spread over a pool of
    worker processes (one torch thread each, as many workers as the process may
    use, at most 16).  For each sampled atom the oracle runs its energy+forces
    path as it stands (the central SCS of every atom the frame needs, the MBD
    and local-SCS reverse pass of the atom, the SCS reverse pass of every atom
    whose central polarisability it uses) and reports the time of each pass and
    its atom count.  The complete job needs one of each per atom, so one core
    spends central/atom + pass B + pass C/atom per atom of the job; the pool
    of workers runs that many atoms at once.
    """
    import multiprocessing as mproc
    import oracle
    from workloads import DEFAULT_PARAMS
    prm = oracle.make_params(cut, grid[0], grid[1], n_max=DEFAULT_PARAMS["n_max"], beta=DEFAULT_PARAMS["beta"],
                             damp_d=DEFAULT_PARAMS["damp_d"], r_buf=DEFAULT_PARAMS["r_buf"],
                             r_inner=DEFAULT_PARAMS["r_inner"])
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    sample = sorted(int(x) for x in np.random.Generator(np.random.PCG64(77)).choice(st.n, n_sample, replace=False))
    _BASE.update(st=st, prm=prm)
    t0 = time.perf_counter()
    with mproc.get_context("fork").Pool(workers, initializer=_baseline_worker_init) as pool:
        tms = pool.map(_baseline_task, sample, chunksize=1)
    wall = time.perf_counter() - t0
    per_atom = [t["central_s"] / t["central_atoms"] + t["pass_b_s"] / t["pass_b_atoms"]
                + t["pass_c_s"] / max(1, t["pass_c_atoms"]) for t in tms]
    core_s = float(np.mean(per_atom))
    return {"value": workers / core_s, "unit": "atoms/s", "cores": workers, "kind": "oracle",
            "cpu_model": host_cpu_model(), "host_cpus_visible": os.cpu_count(),
            "sample": (f"energy+forces path of {n_sample} seeded central atoms of the same 1,728-atom box, "
                       f"{workers} worker processes with one thread each ({wall:.1f} s wall); one core spends "
                       f"{core_s:.3f} s per atom of the complete job (central SCS + MBD/SCS reverse pass + "
                       "SCS reverse pass per atom, from the oracle's own pass timings)"),
            "core_s_per_atom": core_s, "wall_s": wall}


def _replay(srv, reqs, arrivals):
    """Submit each request at its arrival time (s from now); latency runs from the
    arrival to the outputs being written on the host."""
    first_batch = srv.stats()["batches"]
    t0 = time.perf_counter()
    tickets, intake = [], []
    for r, ta in zip(reqs, arrivals):
        dt = ta - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        ts = time.perf_counter()
        tickets.append(srv.submit(r))
        intake.append(time.perf_counter() - ts)   # host-side footprint analysis before queueing
    infos = [srv.wait(t) for t in tickets]
    bad = [i["detail"] for i in infos if i["status"] != "LMBD_OK"]
    if bad:
        raise RuntimeError(f"served requests failed: {bad[:3]}")
    lat = np.array([i["t_end"] - i["t_submit"] + d for i, d in zip(infos, intake)])
    t_first = min(i["t_submit"] - d for i, d in zip(infos, intake))
    span = max(i["t_end"] for i in infos) - t_first
    atoms = sum(len(r["pos"]) for r in reqs)
    stats = srv.stats()
    for t in tickets:
        srv.release(t)
    return {"atoms_per_s": atoms / span, "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "span_s": span,
            "batches": int(stats["batches"] - first_batch),
            "mean_requests_per_batch": float(np.mean([i["batch_requests"] for i in infos])),
            "max_concurrent_batches": int(stats["max_concurrent"]), "pool_peak_GB": stats["pool_peak"] / 1e9}


def serve_bench(sweep=False):
    """Serving workload: mixed-precision continuous batching vs one-at-a-time FP64."""
    import paper_2407_06409_amd as P
    from workloads import SPECIES_TABLE, DEFAULT_PARAMS, frequency_grid
    from workloads import configs as C
    grid = frequency_grid(DEFAULT_PARAMS["n_freq"])
    items = C.serving_requests()
    reqs = [dict(pos=it["structure"].pos, species=it["structure"].species, v_ratio=it["structure"].nu,
                 cell=it["structure"].cell, pbc=tuple(int(x) for x in it["structure"].pbc), cutoffs=it["cutoffs"])
            for it in items]
    unit_gaps = np.array([it["arrival"] for it in items])
    mean_atoms = float(np.mean([len(r["pos"]) for r in reqs]))

    def mp(precision):
        return P.MethodParams(omega=grid[0], weight=grid[1], beta=DEFAULT_PARAMS["beta"],
                              damp_d=DEFAULT_PARAMS["damp_d"], r_buf=DEFAULT_PARAMS["r_buf"],
                              r_inner=DEFAULT_PARAMS["r_inner"], n_max=DEFAULT_PARAMS["n_max"], precision=precision)

    served_cfg = dict(n_slots=SERVE_SLOTS, memory_budget=SERVE_POOL, max_batch_atoms=SERVE_BATCH_ATOMS)
    with P.Server(mp("mixed"), SPECIES_TABLE, **served_cfg) as srv:
        t = srv.submit(reqs[0])  # first-use costs (code objects, pool pages) outside the timed runs
        srv.wait(t)
        srv.release(t)
        cap = _replay(srv, reqs, np.zeros(len(reqs)))
        rate = 0.8 * cap["atoms_per_s"] / mean_atoms
        served = _replay(srv, reqs, unit_gaps / rate)
        sweep_out = {}
        if sweep:
            for m in (0.5, 1.0, 1.2):
                sweep_out[str(m)] = _replay(srv, reqs, unit_gaps / (m / 0.8 * rate))
    with P.Server(mp("fp64"), SPECIES_TABLE, n_slots=1, max_batch_requests=1, memory_budget=SERVE_POOL) as srv:
        t = srv.submit(reqs[0])
        srv.wait(t)
        srv.release(t)
        single_cap = _replay(srv, reqs, np.zeros(len(reqs)))
        single = _replay(srv, reqs, unit_gaps / rate)
    out = {"workload": f"{len(reqs)} H/C/N/O requests, 50-5,000 atoms log-uniform (mean {mean_atoms:.0f}), half open "
                       "spheres and half periodic cubes at 1.0 g/cm3, cutoff U[5,6] A, energy+forces, Poisson "
                       "arrivals at 0.8 x the measured mixed capacity",
           "rate_req_per_s": rate, "capacity_mixed_served_atoms_per_s": cap["atoms_per_s"],
           "capacity_fp64_one_at_a_time_atoms_per_s": single_cap["atoms_per_s"],
           "server": {"n_slots": SERVE_SLOTS, "pool_GB": SERVE_POOL / 1e9, "max_batch_atoms": SERVE_BATCH_ATOMS},
           "mixed_served": served, "fp64_one_at_a_time": single,
           "capacity_ratio": cap["atoms_per_s"] / single_cap["atoms_per_s"]}
    if sweep:
        out["rate_sweep_mixed_served"] = sweep_out
    return out


def mixed_large(args, P, mp):
    """The 13,824-atom carbon box (2.0 g/cm^3, 6 A) in mixed precision, energy+forces:
    atoms/s and ms per step with inputs on the device, and the error of every
    atom's energy and force against the FP64 path on the same GPU (one FP64 step)
    and of the sampled energies against the stored oracle values."""
    import torch
    from workloads import SPECIES_TABLE
    from workloads import configs as C
    st, cut = C.config_mixed_pbc()
    dev = torch.device("cuda:0")
    pos = torch.as_tensor(st.pos, dtype=torch.float64, device=dev)
    sp = torch.as_tensor(st.species, dtype=torch.int32, device=dev)
    nu = torch.as_tensor(st.nu, dtype=torch.float64, device=dev)
    ctx = P.Context(0)
    ctx.set_profiling(True)
    stream = torch.cuda.current_stream(dev)
    mixed = dataclasses.replace(mp, precision="mixed")

    def run(params):
        return P.compute(pos, sp, nu, cutoffs=cut, params=params, species_table=SPECIES_TABLE, cell=st.cell,
                         forces=True, ctx=ctx, stream=stream)

    steps = max(1, min(args.steps, 5))
    for _ in range(max(1, min(args.warmup, 2))):
        run(mixed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        om = run(mixed)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    stg = dict(ctx.stage_times())
    ref = run(mp)   # FP64, same inputs
    torch.cuda.synchronize()
    de = (om["energies"] - ref["energies"]).abs()
    df = (om["forces"] - ref["forces"]).abs()
    rec = {"workload": f"lMBD energy+forces, {st.n} C atoms periodic 2.0 g/cm3, cutoff {cut['r_scs']} A, mixed",
           "value": st.n * steps / el, "unit": "atoms/s", "ms_per_step": el / steps * 1e3, "steps": steps,
           "dtype": "f32 matrices/GEMMs on MFMA, f64 refinement and accumulation",
           "max_abs_dE_vs_fp64_eV_per_atom": float(de.max()), "mean_abs_dE_vs_fp64_eV_per_atom": float(de.mean()),
           "max_abs_dF_vs_fp64_eV_per_A": float(df.max()), "mean_abs_dF_vs_fp64_eV_per_A": float(df.mean()),
           "stages_ms": stg}
    gold = os.path.join(ROOT, "tests", "golden", "oracle_fullsize.json")
    if os.path.exists(gold):
        g = json.load(open(gold))["C13824_pbc"]["energies"]
        e = om["energies"].cpu().numpy()
        rec["max_abs_dE_vs_oracle_sampled_eV_per_atom"] = float(np.abs(e[g["atoms"]] - np.array(g["energies_eV"])).max())
        rec["oracle_sampled_atoms"] = len(g["atoms"])
    ctx.close()
    del ref, om
    torch.cuda.empty_cache()
    return rec


SERVE_SLOTS = 3
SERVE_POOL = 96 << 30
SERVE_BATCH_ATOMS = 8192


def summarize(kind, d, workload):
    """Markdown summary of rocprofv3 output (kernel stats, or FETCH/WRITE counters)."""
    import csv
    import glob

    def one_in(dd, pattern):
        f = sorted(glob.glob(os.path.join(dd, "**", pattern), recursive=True))
        if not f:
            sys.exit(f"no {pattern} under {dd}")
        return list(csv.DictReader(open(f[0])))

    def one(pattern):
        return one_in(d, pattern)

    if kind == "stats":
        rows = one("*kernel_stats.csv")
        out = [f"| kernel | calls | avg ms | share |", "|---|---|---|---|"]
        for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
            out.append(f"| `{r['Name'][:72]}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.3f} | "
                       f"{float(r['Percentage']):.1f}% |")
        return "\n".join(out)
    if kind.startswith("mfma:"):
        # kind = "mfma:<dir>[:<dir> ...]": every counter of the runs, averaged per dispatch, for the
        # factorisation and MBD kernels; MOPS counters are in units of 512 FLOP
        rows = []
        for dd in kind.split(":")[1:]:
            rows += one_in(dd, "*counter_collection.csv")
        out = ["| kernel | counter | mean per dispatch | dispatches |", "|---|---|---|---|"]
        for kn in ("k_scs_factor", "k_mbd"):
            by = {}
            for r in rows:
                if kn in r["Kernel_Name"]:
                    key = (r["Kernel_Name"].split("(")[0].replace("void ", ""), r["Counter_Name"])
                    by.setdefault(key, []).append(float(r["Counter_Value"]))
            for (name, cn), v in sorted(by.items()):
                out.append(f"| `{name}` | {cn} | {np.mean(v):.6g} | {len(v)} |")
        return "\n".join(out)
    # counters: kind = "pmc:<fetch dir>:<write dir>"
    _, dfetch, dwrite = kind.split(":")
    res = {}
    for counter, dd in (("FETCH_SIZE", dfetch), ("WRITE_SIZE", dwrite)):
        d = dd
        rows = [r for r in one("*counter_collection.csv") if r["Counter_Name"] == counter]
        copy = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
        ref = max(copy) if copy else float("nan")
        fac = [float(r["Counter_Value"]) for r in rows if "k_scs_factor" in r["Kernel_Name"]]
        res[counter] = (ref, fac[0] if fac else float("nan"))
    copy_kib = 1024.0 * 1024.0   # the 1 GiB calibration copy (bench.py --calibrate-copy 1024)
    f_fetch = copy_kib / res["FETCH_SIZE"][0]
    f_write = copy_kib / res["WRITE_SIZE"][0]
    hbm = (res["FETCH_SIZE"][1] * f_fetch + res["WRITE_SIZE"][1] * f_write) * 1024.0
    lines = [f"| counter | 1 GiB copy reads (KiB) | calibration factor | k_scs_factor<double> (KiB) | calibrated GB |",
             "|---|---|---|---|---|",
             f"| FETCH_SIZE | {res['FETCH_SIZE'][0]:.0f} | {f_fetch:.4f} | {res['FETCH_SIZE'][1]:.4g} | "
             f"{res['FETCH_SIZE'][1] * f_fetch * 1024 / 1e9:.2f} |",
             f"| WRITE_SIZE | {res['WRITE_SIZE'][0]:.0f} | {f_write:.4f} | {res['WRITE_SIZE'][1]:.4g} | "
             f"{res['WRITE_SIZE'][1] * f_write * 1024 / 1e9:.2f} |",
             "", f"- hbm_bytes_per_launch: `{hbm:.6g}`",
             f"- source_digest: `{source_digest(FACTOR_SOURCES)}`"]
    return "\n".join(lines)


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize":
        print(summarize(sys.argv[2], sys.argv[3] if len(sys.argv) > 3 else ".", ""))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--workload", default="plain", choices=["plain", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving replay")
    ap.add_argument("--serve-sweep", action="store_true", help="also replay at 0.5/1.0/1.2 x the rate")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision timing of the workload")
    ap.add_argument("--no-two-radius", action="store_true",
                    help="skip the timing of the two-radius regime (sparse and dense MBD products)")
    ap.add_argument("--no-two-point", action="store_true",
                    help="skip the timing of the two-point Lorentzian SCS frequency model")
    ap.add_argument("--no-production-radii", action="store_true",
                    help="skip the timing of the production two-radius settings (10 + 8 A)")
    ap.add_argument("--no-fit", action="store_true",
                    help="skip the timing of the eigenvalue-bounded fitted coefficients")
    ap.add_argument("--no-paper-forces", action="store_true",
                    help="skip the timing of the approximate forces of Sec. III.D")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run one plain device copy of MIB MiB (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU design is "
              "documented but not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    from workloads import SPECIES_TABLE, DEFAULT_PARAMS, frequency_grid
    from workloads import configs as C
    from workloads.configs import OMEGA_REF
    import paper_2407_06409_amd as P

    if args.workload == "plain":
        st, cut = C.config_plain_pbc()
    else:
        st, cut = C.config_mixed_pbc()
    grid = frequency_grid(DEFAULT_PARAMS["n_freq"])
    mp = P.MethodParams(omega=grid[0], weight=grid[1], beta=DEFAULT_PARAMS["beta"], damp_d=DEFAULT_PARAMS["damp_d"],
                        r_buf=DEFAULT_PARAMS["r_buf"], r_inner=DEFAULT_PARAMS["r_inner"],
                        n_max=DEFAULT_PARAMS["n_max"], precision=args.precision)
    dev = torch.device("cuda:0")
    pos = torch.as_tensor(st.pos, dtype=torch.float64, device=dev)
    sp = torch.as_tensor(st.species, dtype=torch.int32, device=dev)
    nu = torch.as_tensor(st.nu, dtype=torch.float64, device=dev)
    ctx = P.Context(0)
    ctx.set_profiling(True)
    stream = torch.cuda.current_stream(dev)

    def step():
        return P.compute(pos, sp, nu, cutoffs=cut, params=mp, species_table=SPECIES_TABLE, cell=st.cell,
                         forces=True, ctx=ctx, stream=stream)

    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy * (1 << 20) // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    lat, stages = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        out = step()
        lat.append(time.perf_counter() - ts)
        stages.append(ctx.stage_times())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = st.n * args.steps / elapsed
    stage_ms = {k: float(np.mean([s[k] for s in stages])) for k in stages[0]}

    nq, nw, n_max = len(grid[0]), len(grid[0]) + 1, DEFAULT_PARAMS["n_max"]
    n1 = neighbour_counts(st, cut["r_scs"])
    nK = neighbour_counts(st, cut["r_nbr"])
    # the forward substitution of X = B~^-1 d is carried by the factorisation and
    # the backward one runs in the same kernel, as does the mixed path's refinement
    # (residual and forward + backward correction solve), none of them counted
    flops = {
        "scs_assemble_factor_solve": scs_factor_flops(n1, nw),   # the factorisation's FLOPs only
        "mbd": mbd_flops(nK, nq, n_max, True),
        "scs_lambda": scs_solve_flops(n1, nw, 2),
    }
    peak = PEAK_FP64_TFLOPS if args.precision == "fp64" else PEAK_FP32_TFLOPS
    stage_tflops = {k: flops[k] / (stage_ms[k] * 1e-3) / 1e12 for k in flops if stage_ms.get(k, 0) > 0}
    dom = max(flops, key=lambda k: stage_ms.get(k, 0.0))   # the longest kernel with a dense-algebra count
    ms = stage_ms[dom]
    achieved = flops[dom] / (ms * 1e-3) / 1e12
    traffic = stored_traffic() if (dom == "scs_assemble_factor_solve" and args.precision == "fp64" and args.workload == "plain") else None
    roofline = {"bound": "mfma", "kernel": dom, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": traffic,
                "algorithmic_flops_per_launch": flops[dom], "avg_launch_ms": ms,
                "flops_counted": ("1/3 N^3 per matrix (the launch also assembles B~ and solves for X, "
                                  "which is not counted)" if dom == "scs_assemble_factor_solve"
                                  else "dense algebra of the stage"),
                "traffic_unit": "bytes of HBM traffic per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "stage_tflops": stage_tflops}

    line = {
        "metric": METRIC, "value": value, "unit": "atoms/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"lMBD energy+forces, {st.n} C atoms periodic 2.0 g/cm3, cutoff "
                               f"{cut['r_scs']} A, {nq} GL nodes, n_max {n_max}, {args.precision}",
                   "n_atoms": st.n, "cutoff_A": cut["r_scs"], "n_freq": nq, "n_max": n_max,
                   "precision": args.precision},
        "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "stages_ms": stage_ms, "roofline": roofline,
        "mean_n1": float(n1.mean()), "energy_eV": float(out["energies"].sum().item()),
    }
    def time_params(params, cutoffs=None):
        """Atoms/s, ms per step, the last outputs and stage times of `steps` timed calls."""
        def run():
            return P.compute(pos, sp, nu, cutoffs=cutoffs or cut, params=params, species_table=SPECIES_TABLE,
                             cell=st.cell, forces=True, ctx=ctx, stream=stream)
        for _ in range(args.warmup):
            o = run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            o = run()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        return st.n * args.steps / el, el / args.steps * 1e3, o, dict(ctx.stage_times())

    def max_diff(a, b, key):
        return float((a[key] - b[key]).abs().max())

    if not args.no_mixed and args.precision == "fp64":
        v, msps, om, stg = time_params(dataclasses.replace(mp, precision="mixed"))
        line["mixed"] = {"value": v, "unit": "atoms/s", "ms_per_step": msps,
                         "dtype": "f32 matrices/GEMMs on MFMA, f64 refinement and accumulation",
                         "max_abs_dE_vs_fp64_eV_per_atom": max_diff(om, out, "energies"),
                         "max_abs_dF_vs_fp64_eV_per_A": max_diff(om, out, "forces"),
                         "stages_ms": stg}   # of the last mixed step
    if not args.no_two_point and args.precision == "fp64":
        # the paper's two-point Lorentzian SCS frequency model: 2 SCS solves per atom instead of 13
        tp = {"omega_ref_Ha": OMEGA_REF,
              "model": "SCS at 0 and omega_ref, Lorentzian alpha~(omega) at the nodes (Sec. III.C)"}
        o64 = None
        for prec in ("fp64", "mixed"):
            v, msps, o, stg = time_params(dataclasses.replace(mp, precision=prec, scs_freq="lorentz",
                                                              omega_ref=OMEGA_REF))
            rec = {"value": v, "unit": "atoms/s", "ms_per_step": msps, "stages_ms": stg,
                   "max_abs_dE_vs_exact_treatment_eV_per_atom": max_diff(o, out, "energies"),
                   "mean_abs_dE_vs_exact_treatment_eV_per_atom":
                       float((o["energies"] - out["energies"]).abs().mean()),
                   "max_abs_dF_vs_exact_treatment_eV_per_A": max_diff(o, out, "forces")}
            if prec == "fp64":
                o64 = o
            else:
                rec["max_abs_dE_vs_fp64_eV_per_atom"] = max_diff(o, o64, "energies")
                rec["max_abs_dF_vs_fp64_eV_per_A"] = max_diff(o, o64, "forces")
            tp[prec] = rec
        line["two_point_scs"] = tp
    if not args.no_two_radius and args.precision == "fp64":
        # the two-radius regime of Sec. III.A on the same box: K = B(r_MBD,1 + r_MBD,2)
        cut2 = dict(r_scs=cut["r_scs"], r_nbr=9.0, r_mbd1=6.0, r_mbd2=3.0)
        tr = {"cutoffs_A": cut2, "mean_nK": float(neighbour_counts(st, cut2["r_nbr"]).mean())}
        for mode in ("auto", "dense"):
            ctx.set_mbd_product(mode)
            v, msps, o, stg = time_params(mp, cut2)
            tr["sparse" if mode == "auto" else "dense"] = {"value": v, "unit": "atoms/s", "ms_per_step": msps,
                                                           "stages_ms": stg}
        ctx.set_mbd_product("auto")
        line["two_radius"] = tr
    if not args.no_production_radii and args.precision == "fp64" and args.workload == "plain":
        # Sec. III.A/IV production radii: r_MBD,1 = 10, r_MBD,2 = 8, K = B(18 A) with periodic images
        cut3 = dict(r_scs=cut["r_scs"], r_nbr=18.0, r_mbd1=10.0, r_mbd2=8.0)
        pr = {"cutoffs_A": cut3, "mean_nK": float(neighbour_counts(st, cut3["r_nbr"]).mean()),
              "mean_sites_within_r_mbd2": float(neighbour_counts(st, cut3["r_mbd2"]).mean()),
              "form": "sparse MBD products with the per-site arrays in the workspace"}
        ctx3 = P.Context(0)
        ctx3.set_profiling(True)
        steps3 = min(args.steps, 3)
        for prec in ("fp64", "mixed"):
            prm3 = dataclasses.replace(mp, precision=prec)

            def run3():
                return P.compute(pos, sp, nu, cutoffs=cut3, params=prm3, species_table=SPECIES_TABLE,
                                 cell=st.cell, forces=True, ctx=ctx3, stream=stream)
            run3()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps3):
                o3 = run3()
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            rec = {"value": st.n * steps3 / el, "unit": "atoms/s", "ms_per_step": el / steps3 * 1e3,
                   "steps": steps3, "stages_ms": dict(ctx3.stage_times())}
            if prec == "fp64":
                o3_64 = o3
            else:
                rec["max_abs_dE_vs_fp64_eV_per_atom"] = max_diff(o3, o3_64, "energies")
                rec["max_abs_dF_vs_fp64_eV_per_A"] = max_diff(o3, o3_64, "forces")
            pr[prec] = rec
        pr["energy_eV_per_atom_mean"] = float(o3_64["energies"].mean())
        del o3, o3_64
        # the paper's larger production radii on smaller boxes of the same carbon (K of
        # about 6,600 and 16,500 sites with periodic images)
        larger = {}
        for label, nb, seed, cutL in (("C216_15p10A", 216, 41, dict(r_scs=cut["r_scs"], r_nbr=25.0, r_mbd1=15.0, r_mbd2=10.0)),
                                      ("C64_20p14A", 64, 43, dict(r_scs=cut["r_scs"], r_nbr=34.0, r_mbd1=20.0, r_mbd2=14.0))):
            stL = C.carbon_box(nb, seed, g_cm3=2.0)
            posL = torch.as_tensor(stL.pos, dtype=torch.float64, device=dev)
            spL = torch.as_tensor(stL.species, dtype=torch.int32, device=dev)
            nuL = torch.as_tensor(stL.nu, dtype=torch.float64, device=dev)
            recL = {"cutoffs_A": cutL, "mean_nK": float(neighbour_counts(stL, cutL["r_nbr"]).mean())}
            for prec in ("fp64", "mixed"):
                prmL = dataclasses.replace(mp, precision=prec)

                def runL():
                    return P.compute(posL, spL, nuL, cutoffs=cutL, params=prmL, species_table=SPECIES_TABLE,
                                     cell=stL.cell, forces=True, ctx=ctx3, stream=stream)
                runL()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                oL = runL()
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                recL[prec] = {"value": stL.n / el, "unit": "atoms/s", "ms_per_step": el * 1e3, "steps": 1}
                if prec == "fp64":
                    oL64 = oL
                else:
                    recL[prec]["max_abs_dE_vs_fp64_eV_per_atom"] = max_diff(oL, oL64, "energies")
                    recL[prec]["max_abs_dF_vs_fp64_eV_per_A"] = max_diff(oL, oL64, "forces")
            larger[label] = recL
            del oL, oL64
        pr["larger_radii"] = larger
        ctx3.close()
        line["production_radii"] = pr
    if not args.no_fit and args.precision == "fp64":
        # Sec. III.A: per atom and node, c_n fitted to ln(1 - x) on the Lanczos bounds of G~
        fit = {"lanczos_steps": mp.lanczos_steps,
               "model": "least-squares polynomial of ln(1 - x) of degree n_max on the Lanczos spectrum "
                        "bounds of each atom and node (Sec. III.A); forces with the coefficients held fixed"}
        o64 = None
        for prec in ("fp64", "mixed"):
            v, msps, o, stg = time_params(dataclasses.replace(mp, precision=prec, cn_mode="fit"))
            rec = {"value": v, "unit": "atoms/s", "ms_per_step": msps, "stages_ms": stg,
                   "max_abs_dE_vs_series_eV_per_atom": max_diff(o, out, "energies"),
                   "mean_abs_dE_vs_series_eV_per_atom": float((o["energies"] - out["energies"]).abs().mean())}
            if prec == "fp64":
                o64 = o
            else:
                rec["max_abs_dE_vs_fp64_eV_per_atom"] = max_diff(o, o64, "energies")
                rec["max_abs_dF_vs_fp64_eV_per_A"] = max_diff(o, o64, "forces")
            fit[prec] = rec
        spec = P.compute(pos, sp, nu, cutoffs=cut, params=dataclasses.replace(mp, cn_mode="fit"),
                         species_table=SPECIES_TABLE, cell=st.cell, forces=False, ctx=ctx, stream=stream,
                         want_spectrum=True)["spectrum"]
        fit["spectrum_bounds"] = {"min_lambda_min": float(spec[..., 0].min()),
                                  "max_lambda_max": float(spec[..., 1].max())}
        line["fitted_cn"] = fit
    if not args.no_paper_forces and args.precision == "fp64":
        # Sec. III.D: each atom's force from its own neighbourhood, central polarisabilities fixed
        pf = {"model": "approximate forces of Sec. III.D (Eqs. full-pol-grad, cent-appr-step, cent-appr)"}
        for prec in ("fp64", "mixed"):
            v, msps, o, stg = time_params(dataclasses.replace(mp, precision=prec, force_model="paper"))
            d = (o["forces"] - out["forces"]).norm(dim=1)
            pf[prec] = {"value": v, "unit": "atoms/s", "ms_per_step": msps, "stages_ms": stg,
                        "max_abs_dF_vs_exact_eV_per_A": max_diff(o, out, "forces"),
                        "rms_dF_vs_exact_eV_per_A": float(d.pow(2).mean().sqrt()),
                        "rms_F_exact_eV_per_A": float(out["forces"].norm(dim=1).pow(2).mean().sqrt())}
        line["paper_forces"] = pf
    if not args.no_mixed and args.precision == "fp64" and args.workload == "plain":
        line["mixed_c13824"] = mixed_large(args, P, mp)
    if not args.no_serve:
        line["served"] = serve_bench(args.serve_sweep)
    if not args.no_cpu_baseline and args.workload == "plain":
        line["cpu_baseline"] = cpu_baseline(st, cut, grid)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
