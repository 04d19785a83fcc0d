"""Benchmark of the TBPM propagation path on one MI355X.

Default workload: graphene 4096 x 4096 cells (33,554,432 orbitals) with
Anderson disorder uniform in [-0.5, 0.5] eV, complex128 throughout, rescale
9 eV, 1024 time steps, random-phase vectors processed one at a time.  One
benchmark step is one whole pass of the path for one vector: coefficients,
random-phase state, 1024 time steps of 19 fused Chebyshev terms with the
correlation sums, the copy of C(t) to the host and the DOS transform.

Prints one JSON line: the throughput in Hamiltonian-nnz x Chebyshev-terms per
second, the roofline of the dominant kernel (the middle Chebyshev term),
timed live with HIP events on its launch stream, and the CPU oracle timed on
a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E
# sources that decide the HBM traffic of the timed kernels: the kernels and
# the row order of the patch format
TRAFFIC_SOURCES = [os.path.join(ROOT, "paper_2509_26309_amd", "csrc", f) for f in ("tbpm_kernels.hip", "tbpm_patch.cpp")]

WORKLOADS = {
    # name: (generator, kwargs, rescale, dtype, block, num_time_steps, vectors per step, cycle of vectors, seed)
    "graphene4096_disorder_c128": dict(
        lattice="graphene", dims=(4096, 4096), disorder_w=1.0, lattice_seed=2, rescale=9.0, dtype="c128",
        block=1, nt=1024, vectors=1, cycle=4, seed=2,
        text="graphene 4096x4096 cells (33.5M orbitals), t=-2.7 eV, Anderson disorder U[-0.5,0.5] eV, "
             "complex128 throughout, rescale 9 eV, 1024 time steps, 4 random vectors one at a time"),
    "graphene64_c128": dict(
        lattice="graphene", dims=(64, 64), disorder_w=0.0, lattice_seed=0, rescale=9.0, dtype="c128",
        block=1, nt=256, vectors=1, cycle=1, seed=1,
        text="graphene 64x64 cells (8192 orbitals), t=-2.7 eV, complex128, CSR input (stored in the library's "
             "format), rescale 9 eV, 256 steps, 1 vector; launch-bound: time steps replayed from HIP graphs"),
    "honeycomb7000_3nn_vac_c64_b8": dict(
        lattice="honeycomb3", dims=(7000, 7000), vacancy_p=0.01, lattice_seed=5, rescale=10.0, dtype="c64",
        block=8, nt=4096, vectors=8, cycle=1, seed=5, ldos_sites=1024, sites_seed=55,
        text="honeycomb 7000x7000 cells, 1st-3rd neighbours (-2.7, -0.2, -0.18 eV), 1% random vacancies "
             "(~97M orbitals, ~12 nnz/row), complex64 ELL, 8-vector block, 4096 steps, LDOS at 1024 sites"),
    "bilayer2048_disorder_c64_b16": dict(
        lattice="bilayer", dims=(2048, 2048), disorder_w=1.0, lattice_seed=3, rescale=9.0, dtype="c64",
        block=16, nt=2048, vectors=16, cycle=1, seed=3,
        text="AB bilayer graphene 2048x2048 cells (16.8M orbitals), gamma1=0.39 eV, W=1 eV, complex64 "
             "SpMM of 16 vectors, FP64 coefficients and C(t) sums, 2048 steps"),
}


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def make_lattice(w):
    import tb_inputs as ti
    la, lb = w["dims"]
    if w["lattice"] == "graphene":
        return ti.graphene(la, lb, disorder_w=w["disorder_w"], seed=w["lattice_seed"])
    if w["lattice"] == "bilayer":
        return ti.bilayer(la, lb, disorder_w=w["disorder_w"], seed=w["lattice_seed"])
    if w["lattice"] == "honeycomb3":
        return ti.honeycomb3(la, lb, vacancy_p=w["vacancy_p"], seed=w["lattice_seed"])
    raise ValueError(w["lattice"])


def h_row_values_bytes(info, sv):
    """Bytes per row for the values of H: w values, or with a value table
    (patch format) the row's one-byte indices in ceil(w/4) 4-byte words plus
    the diagonal when it is kept per row (table_diag 1: a value, 2: its real
    part)."""
    w = info["ell_w"]
    if info.get("table_used"):
        return 4 * ((w + 3) // 4) + {0: 0, 1: sv, 2: sv // 2}[int(info.get("table_diag", 0))]
    return w * sv


def algorithmic_bytes_per_launch(info, n, B, dtype, clenshaw=False):
    """Bytes one launch of the middle-term kernel must move.
    Forward recurrence (the paper's): single term: H once, and per element of
    the B vectors a gathered read of x, read+write of y and of out
    (5 accesses); fused pair (patch format, one vector): H once for two
    terms with 2-byte patch-local columns, reads of x_{m-1}, y_{m-2}, writes
    of y_m, x_{m+1}, and one read+write of out (6 accesses).
    Clenshaw's backward recurrence b_m = c_m psi + (2/rho) H b_m+1 - b_m+2:
    single term: a gathered read of b_m+1, reads of b_m+2 and psi, a write of
    b_m (4 accesses); fused pair: reads of b_m+1, b_m+2 and psi, writes of
    b_m, b_m-1 (5 accesses).
    H's values: see h_row_values_bytes (value table of the patch format)."""
    sv = 16 if dtype == "c128" else 8
    # patch-local 2-byte column indices, four to an 8-byte word: 8 ceil(w/4) bytes a row
    lcol = 8 * ((info["ell_w"] + 3) // 4)
    # fused pairs: one vector, or (forward recurrence) complex64 blocks that the library pairs
    pairs = info["format"] == 3 and (B == 1 or (info.get("block_pairs") and not clenshaw))
    if pairs:
        h = n * (lcol + h_row_values_bytes(info, sv))
    elif info["format"] == 3 and dtype == "c64" and B in (8, 16):
        # the staged complex64 SpMM on patch-reordered ELL
        h = n * (lcol + h_row_values_bytes(info, sv))
    elif info["format"] in (1, 3):    # ELL: w slots of (value, column) per row
        w = info["ell_w"]
        w = info["ell_w"]
        h = w * n * (sv + 4)
    else:
        h = info["nnz"] * (sv + 4) + (n + 1) * (8 if info["nnz"] >= 2 ** 31 - 1 else 4)
    k = 1 if clenshaw else 0
    if pairs:
        return h + (6 - k) * sv * n * B, h, 2
    return h + (5 - k) * sv * n * B, h, 1


def traffic_source_hash() -> str:
    return hashlib.sha256(b"".join(open(f, "rb").read() for f in TRAFFIC_SOURCES)).hexdigest()


def bytes_model_text(info, B, terms_per_launch, clenshaw, route):
    """What `algorithmic_bytes_per_launch` counts, in words."""
    staged = info["format"] == 3 and B in (8, 16)
    if info.get("table_used") and (B == 1 or staged):
        vals = ("4 ceil(w/4) bytes of one-byte value indices" +
                {0: "", 1: " + s_val for the row's diagonal",
                 2: " + s_val / 2 for the real part of the row's diagonal"}[int(info.get("table_diag", 0))] +
                " per row (value table)")
        h = "H once: n (8 ceil(w/4) + " + vals + "), 2-byte patch-local columns four to a word"
    else:
        h = ("H once: n (8 ceil(w/4) + w s_val) bytes (2-byte patch-local columns four to a word, values)"
             if info["format"] == 3 and (B == 1 or staged) else
             "H once: w n (s_val + 4) bytes (slot-major ELL)" if info["format"] in (1, 3)
             else "H once: nnz (s_val + 4) + (n + 1) s_rowptr bytes (CSR)")
    if route in ("moments", "sites"):
        v = ("4 vector passes for two products (reads of p_m, p_m-1; writes of p_m+1, p_m+2)"
             if terms_per_launch == 2 else "3 vector passes (gathered p_m, read and write of p_m-1 -> p_m+1)")
    elif terms_per_launch == 2:
        v = ("5 vector passes for two products (reads of b_m+1, b_m+2, psi; writes of b_m, b_m-1)" if clenshaw
             else "6 vector passes for two terms (reads of x_m-1, y_m-2; writes of y_m, x_m+1; out read and "
                  "written once)")
    else:
        v = ("4 vector passes (gathered b_m+1, reads of b_m+2 and psi, write of b_m)" if clenshaw
             else "5 vector passes (gathered x, y read and written, out read and written)")
    return f"{h} + {v}, each pass s_x n B bytes (B = {B})"


def read_traffic(kernel_tag: str, workload: str, series: str):
    """HBM bytes per launch from the committed counter summary, or None when
    absent, taken on different kernel or patch-planner sources, or taken with
    the other series evaluation (the single-term kernels take it as a run-time
    flag, so the kernel name alone does not tell the two apart)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel_tag}_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != traffic_source_hash() or vals.get("series") != series:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def host_cpu():
    """CPU model, logical CPUs, physical cores and sockets of this host (from /proc/cpuinfo),
    and the CPUs this process may run on."""
    model, cores, sockets, logical = None, set(), set(), 0
    phys = core = None
    try:
        for line in open("/proc/cpuinfo"):
            k, _, v = line.partition(":")
            k, v = k.strip(), v.strip()
            if k == "processor":
                logical += 1
            elif k == "model name" and model is None:
                model = v
            elif k == "physical id":
                phys = v
                sockets.add(v)
            elif k == "core id":
                core = v
            elif not k and phys is not None and core is not None:
                cores.add((phys, core))
                phys = core = None
        if phys is not None and core is not None:
            cores.add((phys, core))
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"cpu_model": model, "logical_cpus": logical or os.cpu_count(), "physical_cores": len(cores) or None,
            "sockets": len(sockets) or None, "cpus_usable_by_process": usable}


def copy_calibration(mib: int, reps: int) -> None:
    """A plain device-to-device copy of exactly `mib` MiB, `reps` times: run under
    rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE), it gives the scale between
    those counters and the true bytes of a kernel's HBM traffic."""
    import torch
    n = mib << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_mib": mib, "reps": reps}), flush=True)


def cpu_baseline(lat, w, target_s: float, gpu_corr0=None):
    """The oracle (as it is) on a bounded sample: vector 0 of the workload for
    as many time steps as fit in about target_s seconds."""
    import numpy as np
    import oracle
    psi0 = oracle.random_state(lat.n, w["seed"], 0)
    # per-step cost from the difference of a 2- and a 1-step run (set-up excluded)
    t0 = time.perf_counter()
    res = oracle.propagate(lat, psi0, rescale=w["rescale"], num_steps=1)
    t1 = time.perf_counter()
    res = oracle.propagate(lat, psi0, rescale=w["rescale"], num_steps=2)
    t2 = time.perf_counter()
    one = max((t2 - t1) - (t1 - t0), 0.25 * (t2 - t1), 1e-9)
    el = t2 - t1
    steps = max(2, min(w["nt"], int(target_s / one)))
    if steps > 2:
        t0 = time.perf_counter()
        res = oracle.propagate(lat, psi0, rescale=w["rescale"], num_steps=steps)
        el = time.perf_counter() - t0
    terms = res.num_terms - 1
    threads = oracle.num_threads()
    out = {"value": lat.nnz * terms * steps / el, "unit": "nnz*terms/s", "cores": threads,
           "kind": "oracle",
           "sample": f"vector 0 of the workload, {steps} time step(s) of {terms} terms, {el:.1f} s "
                     f"(FP64 CSR, OpenMP over rows, {threads} threads)",
           "host": host_cpu()}
    # the same oracle on one thread, over a shorter sample (a fifth of the budget)
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.propagate(lat, psi0, rescale=w["rescale"], num_steps=1)
        one1 = time.perf_counter() - t0
        s1 = max(1, min(steps, int(0.2 * target_s / max(one1, 1e-9))))
        t0 = time.perf_counter()
        oracle.propagate(lat, psi0, rescale=w["rescale"], num_steps=s1)
        el1 = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(threads)
    out["value_1thread"] = lat.nnz * terms * s1 / el1
    out["sample_1thread"] = f"vector 0, {s1} time step(s), {el1:.1f} s on 1 thread"
    if gpu_corr0 is not None:
        k = min(steps, gpu_corr0.size - 1)
        out["max_abs_dC_vs_gpu"] = float(np.abs(gpu_corr0[:k + 1] - res.corr[:k + 1]).max())
        if k >= 2:
            # the same windowed transform of both C(t) prefixes (N_t = k): the DOS error
            # that the GPU's C(t) carries over the sampled time range
            _, d_gpu = oracle.dos(gpu_corr0[:k + 1], w["rescale"])
            _, d_ref = oracle.dos(res.corr[:k + 1], w["rescale"])
            out["max_abs_dDOS_vs_gpu"] = float(np.abs(d_gpu - d_ref).max())
            # integrated error: sum_j |d_gpu - d_ref| times the energy spacing rho / N_t
            out["sum_abs_dDOS_dE_vs_gpu"] = float(np.abs(d_gpu - d_ref).sum() * w["rescale"] / k)
            out["dos_steps_compared"] = int(k)
    return out


# reduced instances of the complex64 workloads' generators, run for the workloads'
# full step counts: (generator, dims, lattice kwargs, format the library picks)
FULL_LENGTH_CHECK = {
    "bilayer2048_disorder_c64_b16": ("bilayer", (128, 128), {"disorder_w": 1.0, "seed": 3}),
    "honeycomb7000_3nn_vac_c64_b8": ("honeycomb3", (96, 96), {"vacancy_p": 0.01, "seed": 5}),
}


def full_length_check(ctx, tbpm, name, w):
    """The complex64 path on a reduced lattice of the workload's generator for
    the workload's full number of steps, in the workload's block width:
    max |dC| of vector 0 against the FP64 oracle over all N_t + 1 steps, and
    the DOS error of that C(t)."""
    import numpy as np
    import oracle
    import tb_inputs as ti
    gen, (la, lb), kw = FULL_LENGTH_CHECK[name]
    lat = getattr(ti, gen)(la, lb, **kw)
    ham = ctx.build(lat, dtype=tbpm.TBPM_C64)
    try:
        p, _keep = tbpm.make_params(w["rescale"], w["nt"], w["block"], block=w["block"], seed=w["seed"])
        out = tbpm.tbpm_propagate_dos(ctx.handle, ham, p)
        fmt = {0: "CSR", 1: "ELL", 3: "PATCH-ELL"}[tbpm.tbpm_ham_info(ham)["format"]]
    finally:
        tbpm.tbpm_ham_destroy(ham)
    ref = oracle.propagate(lat, oracle.random_state(lat.n, w["seed"], 0), rescale=w["rescale"], num_steps=w["nt"])
    _, d_gpu = oracle.dos(out["corr"][0], w["rescale"])
    _, d_ref = oracle.dos(ref.corr, w["rescale"])
    return {"instance": f"{gen} {la}x{lb} {kw}, {lat.n} orbitals, {fmt}, block {w['block']}, {w['nt']} steps, "
                        f"vector 0", "max_abs_dC": float(np.abs(out["corr"][0] - ref.corr).max()),
            "max_abs_dDOS": float(np.abs(d_gpu - d_ref).max()),
            "max_norm_drift": float(np.abs(out["norms"][0] - 1).max())}


def cpu_baseline_moments(lat, w, target_s: float, gpu_mu0=None, site=None):
    """The oracle's moment recurrence (as it is) on a bounded sample: vector 0
    of the workload (or one site-localised state), as many moments as fit in
    about target_s seconds (one product with H per moment)."""
    import numpy as np
    import oracle
    import tb_inputs as ti
    psi0 = oracle.random_state(lat.n, w["seed"], 0) if site is None else ti.state_from_sites(lat.n, [site])
    t0 = time.perf_counter()
    oracle.moments(lat, psi0, rescale=w["rescale"], num_moments=9)
    one = (time.perf_counter() - t0) / 8
    num = max(4, min(4096, int(target_s / max(one, 1e-9))))
    if gpu_mu0 is not None:
        num = min(num, gpu_mu0.size)
    t0 = time.perf_counter()
    mu = oracle.moments(lat, psi0, rescale=w["rescale"], num_moments=num)
    el = time.perf_counter() - t0
    out = {"value": lat.nnz * (num - 1) / el, "unit": "nnz*terms/s", "cores": oracle.num_threads(),
           "kind": "oracle",
           "sample": f"{'vector 0 of the workload' if site is None else f'site {site}'}, {num} moments by the "
                     f"plain recurrence ({num - 1} products "
                     f"with H), {el:.1f} s (FP64 CSR, OpenMP over rows)"}
    if gpu_mu0 is not None:
        out["max_abs_dmu_vs_gpu"] = float(np.abs(gpu_mu0[:num] - mu).max())
    return out


def serving(args):
    """Serving mix: a Poisson trace of requests submitted at their arrival
    times to the continuous-batching server; latency = completion - arrival.
    Baseline: the same trace replayed one request at a time on the plain FP64
    path (complex128, one vector per block), requests served in arrival order."""
    import numpy as np
    from paper_2509_26309_amd import tbpm
    from tb_inputs.trace import serving_trace, build_lattice

    reqs = serving_trace(num_requests=args.serve_requests, rate=50.0, seed=4, n_max=args.serve_n_max)
    ctx = tbpm.Context(0)
    if args.series == "clenshaw":
        tbpm.tbpm_ctx_set_series(ctx.handle, tbpm.TBPM_SERIES_CLENSHAW)
    terms = len(tbpm.tbpm_coefficients(np.pi)) - 1
    hams, hams64, work = {}, {}, {}
    t = time.perf_counter()
    for r in reqs:
        log(f"serving: building request {r.index}: {r.lattice} {r.orbitals} orbitals")
        lat = build_lattice(r)
        hams[r.index] = ctx.build(lat, dtype=tbpm.TBPM_C64 if r.fp32 else tbpm.TBPM_C128)
        hams64[r.index] = ctx.build(lat, dtype=tbpm.TBPM_C128) if r.fp32 else hams[r.index]
        work[r.index] = lat.nnz * terms * r.time_steps * r.vectors
    log(f"serving: {len(reqs)} requests, matrices built in {time.perf_counter() - t:.1f} s")

    def params(r, block=0):
        return tbpm.make_params(r.rescale, r.time_steps, r.vectors, seed=r.seed, block=block)[0]

    # warm the kernels once
    for r in reqs[:2]:
        tbpm.tbpm_propagate_dos(ctx.handle, hams[r.index], params(r))
    srv = tbpm.tbpm_server_create(ctx.handle, args.serve_budget_gb << 30, args.serve_slots)
    t0 = time.perf_counter()
    tickets = {}
    for r in reqs:
        while time.perf_counter() - t0 < r.arrival:
            time.sleep(0.0005)
        tickets[r.index] = tbpm.tbpm_submit(srv, hams[r.index], params(r))
    lat_s, svc_s, stat = {}, {}, {}
    left = set(tickets)
    while left:
        for i in list(left):
            r = reqs[i]
            st, _, tm, _ = tbpm.tbpm_poll(srv, tickets[i], r.vectors, r.time_steps)
            if st != tbpm.TBPM_PENDING:
                lat_s[i] = tm[2] - tm[0]
                svc_s[i] = tm[2] - tm[1]
                stat[i] = (st, tm)
                left.discard(i)
                log(f"serving: request {i} ({r.orbitals} orbitals, {r.vectors} vectors, {r.time_steps} steps, "
                    f"{'FP32' if r.fp32 else 'FP64'}) done: latency {lat_s[i]:.2f} s, status {st}")
        time.sleep(0.002)
    tbpm.tbpm_server_destroy(srv)
    first = min(v[1][0] for v in stat.values())
    wall = max(v[1][2] for v in stat.values()) - first
    ok = all(v[0] == tbpm.TBPM_OK for v in stat.values())
    lat = np.array([lat_s[i] for i in sorted(lat_s)])
    svc = np.array([svc_s[i] for i in sorted(svc_s)])
    total_work = sum(work.values())
    log(f"serving: mix done in {wall:.1f} s, all ok={ok}")

    # replay: plain FP64 (forward recurrence), one request at a time, in arrival order
    tbpm.tbpm_ctx_set_series(ctx.handle, tbpm.TBPM_SERIES_FORWARD)
    end = 0.0
    rl = []
    busy = 0.0
    for r in reqs:
        t1 = time.perf_counter()
        tbpm.tbpm_propagate_dos(ctx.handle, hams64[r.index], params(r, block=1))
        d = time.perf_counter() - t1
        busy += d
        start = max(r.arrival, end)
        end = start + d
        rl.append(end - r.arrival)
        log(f"serving: replay request {r.index} took {d:.2f} s")
    rl = np.array(rl)
    replay_wall = end - reqs[0].arrival
    log(f"serving: replay busy {busy:.1f} s")
    for i in hams:
        if hams64[i] is not hams[i]:
            tbpm.tbpm_ham_destroy(hams64[i])
        tbpm.tbpm_ham_destroy(hams[i])
    ctx.close()
    line = {
        "metric": "p99 solve latency (serving mix)", "value": float(np.percentile(lat, 99)), "unit": "s",
        "n_gpus": 1, "higher_is_better": False, "data": "synthetic", "dtype": "f32/f64 per request",
        "config": {"workload": "serving_mix", "requests": len(reqs), "rate_per_s": 50.0,
                   "n_range": [1e4, args.serve_n_max], "vectors": [1, 32], "time_steps": [128, 2048],
                   "hbm_budget_gb": args.serve_budget_gb, "slots": args.serve_slots, "series": args.series},
        "serving": {"p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
                    "p50_service_s": float(np.percentile(svc, 50)), "p99_service_s": float(np.percentile(svc, 99)),
                    "wall_s": wall, "throughput_nnz_terms_per_s": total_work / wall, "all_ok": ok},
        "replay_fp64_one_at_a_time": {"p50_latency_s": float(np.percentile(rl, 50)),
                                      "p99_latency_s": float(np.percentile(rl, 99)), "wall_s": replay_wall,
                                      "throughput_nnz_terms_per_s": total_work / busy},
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4, help="timed steps (vectors)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="graphene4096_disorder_c128", choices=sorted(WORKLOADS) + ["serving_mix"])
    ap.add_argument("--serve-requests", type=int, default=20)
    ap.add_argument("--serve-n-max", type=float, default=1e7)
    ap.add_argument("--serve-budget-gb", type=int, default=64)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--time-steps", type=int, default=0, help="override the workload's number of time steps")
    ap.add_argument("--block", type=int, default=0,
                    help="override the workload's vectors per block (the vectors per step stay the workload's)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="CPU oracle sample budget (0: skip)")
    ap.add_argument("--format", default="auto", choices=["auto", "csr", "ell", "patch"],
                    help="device format of H (auto: the library's choice)")
    ap.add_argument("--large-patches", action="store_true", help="2048-row patches for the patch format")
    ap.add_argument("--no-value-table", action="store_true",
                    help="store every entry's value (no value table) in the patch format")
    ap.add_argument("--series", default="forward", choices=["forward", "clenshaw"],
                    help="series evaluation: the paper's forward recurrence (headline) or Clenshaw's backward "
                         "recurrence (a formulation variant, reported on its own line)")
    ap.add_argument("--alloc", default="torch", choices=["torch", "hip"],
                    help="device memory from PyTorch's caching allocator or hipMalloc")
    ap.add_argument("--route", default="propagate",
                    choices=["propagate", "moments", "qe", "wft", "sites", "ac", "dp"],
                    help="propagate: time steps of the Chebyshev series (the path); moments: the same C(t) "
                         "and DOS from Chebyshev moments (a separate formulation, reported on its own line); "
                         "qe: the propagation plus quasi-eigenstates at --qe-energies; wft: the propagation "
                         "plus snapshots of psi(t) every --wft-every steps (one vector per step)")
    ap.add_argument("--qe-energies", default="-2.7,-1.0,-0.5,0.0,0.5,1.0,2.7,5.0",
                    help="energies (eV) of the quasi-eigenstates for --route qe")
    ap.add_argument("--wft-every", type=int, default=128, help="snapshot interval (steps) for --route wft")
    ap.add_argument("--kT", type=float, default=0.02585, help="--route ac/dp: temperature (eV), 300 K default")
    ap.add_argument("--mu", type=float, default=0.0, help="--route ac/dp: chemical potential (eV)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (three times), for scaling the HBM counters")
    ap.add_argument("--sites", type=int, default=0,
                    help="--route sites: exact LDOS (Chebyshev moments of site-localised states) at this many "
                         "sampled orbitals per bench step (0: the workload's LDOS site count, else 16)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the propagation of independent random vectors would shard over "
              "GPUs with one all-reduce of C(t) at the end; only single-GPU runs are supported.",
              file=sys.stderr)
        sys.exit(2)

    if args.calibrate_copy > 0:
        copy_calibration(args.calibrate_copy, 3)
        return
    if args.workload == "serving_mix":
        serving(args)
        return

    import numpy as np
    import torch
    from paper_2509_26309_amd import tbpm

    w = dict(WORKLOADS[args.workload])
    if args.time_steps > 0:
        w["nt"] = args.time_steps
    t = time.perf_counter()
    lat = make_lattice(w)
    log(f"bench: lattice {args.workload} n={lat.n} nnz={lat.nnz} built in {time.perf_counter() - t:.1f} s")

    dtype = tbpm.TBPM_C128 if w["dtype"] == "c128" else tbpm.TBPM_C64
    ctx = tbpm.Context(0, allocator=args.alloc, torch_stream=(args.alloc == "torch"))
    clenshaw = args.series == "clenshaw"
    if clenshaw:
        tbpm.tbpm_ctx_set_series(ctx.handle, tbpm.TBPM_SERIES_CLENSHAW)
    fmt = {"auto": tbpm.TBPM_FMT_AUTO, "csr": tbpm.TBPM_FMT_CSR, "ell": tbpm.TBPM_FMT_ELL,
           "patch": tbpm.TBPM_FMT_PATCH}[args.format]
    t = time.perf_counter()
    bflags = ((tbpm.TBPM_BUILD_LARGE_PATCHES if args.large_patches else 0) |
              (tbpm.TBPM_BUILD_NO_VALUE_TABLE if args.no_value_table else 0))
    ham = ctx.build(lat, dtype=dtype, fmt=fmt, flags=bflags)
    info = tbpm.tbpm_ham_info(ham)
    info["ell_w"] = int(np.diff(lat.row_ptr).max())
    vt = tbpm.tbpm_ham_value_table(ham)
    # the fused pairs use the table with 1024-row patches, the staged complex64 SpMM always
    info["table_used"] = vt["entries"] > 0 and info["format"] == 3 and not (args.large_patches and info["ell_w"] <= 5)
    info["table_diag"] = int(vt["per_row_diagonal"])
    fmt_name = {0: "CSR", 1: "ELL", 3: "PATCH-ELL"}[info["format"]]
    log(f"bench: H on device in {time.perf_counter() - t:.1f} s, format={fmt_name} bytes={info['bytes']}")
    rescale, nt, R, B = w["rescale"], w["nt"], w["vectors"], (args.block or w["block"])
    # complex64 blocks whose middle terms the library applies two to a launch
    info["block_pairs"] = B > 1 and tbpm.tbpm_ham_fused_pairs(ham, B)
    import tb_inputs as ti
    sites = ti.sample_sites(lat.n, w["ldos_sites"], w["sites_seed"]) if w.get("ldos_sites") else None

    num_moments = tbpm.tbpm_moments_needed(nt) if args.route in ("moments", "sites") else 0
    n_sites = args.sites or w.get("ldos_sites", 16)
    if args.route == "sites":
        R = n_sites

    def one_step_sites(i, keep):
        p, _keep = tbpm.make_params(rescale, 0, 1, block=B)
        s_i = ti.sample_sites(lat.n, n_sites, w.get("sites_seed", 55) + i % w["cycle"])
        mu = tbpm.tbpm_site_moments(ctx.handle, ham, p, s_i, num_moments)
        e, d = tbpm.tbpm_kpm_dos(mu[0], rescale, 2 * nt)
        out = {"mu": mu, "sites": s_i}
        if keep is not None:
            keep.append(out)
        return out

    def one_step_moments(i, keep):
        p, _keep = tbpm.make_params(rescale, 0, R, block=B, seed=w["seed"], first_vector=(i % w["cycle"]) * R)
        mu = tbpm.tbpm_chebyshev_moments(ctx.handle, ham, p, num_moments)
        corr = tbpm.tbpm_corr_from_moments(tbpm.tbpm_sample_mean(mu), nt)
        e, d = tbpm.tbpm_dos(corr, rescale)
        out = {"mu": mu, "corr": corr[None, :]}
        if keep is not None:
            keep.append(out)
        return out

    qe_energies = [float(x) for x in args.qe_energies.split(",")]
    wft_steps = list(range(0, nt + 1, max(1, args.wft_every)))
    if args.route in ("qe", "wft") and R != 1:
        log(f"bench: --route {args.route} takes one vector per step; workload {args.workload} has {R}")
        sys.exit(2)

    def one_step_outputs(i, keep):
        p, _keep = tbpm.make_params(rescale, nt, 1, seed=w["seed"], first_vector=i % w["cycle"])
        if args.route == "qe":
            out = tbpm.tbpm_quasi_eigenstates(ctx.handle, ham, p, qe_energies)
            out["qe_norms"] = np.linalg.norm(out.pop("qe"), axis=1)
        else:
            out = tbpm.tbpm_time_evolution(ctx.handle, ham, p, wft_steps)
            out["snapshot_norms"] = np.linalg.norm(out.pop("snapshots"), axis=1)
        e, d = tbpm.tbpm_dos(out["corr"], rescale)
        out["corr"] = out["corr"][None, :]
        if keep is not None:
            keep.append(out)
        return out

    ops = None
    if args.route in ("ac", "dp"):
        t = time.perf_counter()
        if args.route == "ac":
            a_op = ti.current_operator(lat, (1.0, 0.0))
            ops = (ctx.operator(ham, a_op),)
            ops = (ops[0], ops[0])
        else:
            q = (2 * np.pi / (lat.dims[0] * ti.lattices.GRAPHENE_A) * 16, 0.0)
            ops = (ctx.operator(ham, ti.density_operator(lat, q)),
                   ctx.operator(ham, ti.density_operator(lat, (-q[0], -q[1]))))
        fermi_terms = tbpm.tbpm_fermi_coefficients(rescale, args.mu, args.kT).size
        log(f"bench: operators on device in {time.perf_counter() - t:.1f} s; {fermi_terms} Fermi terms")

    def one_step_response(i, keep):
        p, _keep = tbpm.make_params(rescale, nt, 1, seed=w["seed"], first_vector=i % w["cycle"])
        corr = tbpm.tbpm_response_corr(ctx.handle, ham, ops[0], ops[1], p, args.mu, args.kT)
        omegas = np.linspace(0.1, 6.0, 60)
        if args.route == "ac":
            res = tbpm.tbpm_ac_conductivity(corr[0], rescale, args.kT, ti.area_per_orbital(lat), omegas)
        else:
            res = tbpm.tbpm_dyn_polarization(corr[0], rescale, ti.area_per_orbital(lat), omegas)
        out = {"corr": corr, "result": res, "omegas": omegas}
        if keep is not None:
            keep.append(out)
        return out

    def one_step(i, keep):
        if args.route in ("ac", "dp"):
            return one_step_response(i, keep)
        if args.route == "sites":
            return one_step_sites(i, keep)
        if args.route == "moments":
            return one_step_moments(i, keep)
        if args.route in ("qe", "wft"):
            return one_step_outputs(i, keep)
        p, _keep = tbpm.make_params(rescale, nt, R, block=B, seed=w["seed"], first_vector=(i % w["cycle"]) * R,
                                    sites=sites)
        out = tbpm.tbpm_propagate_dos(ctx.handle, ham, p, want_norms=True)
        e, d = tbpm.tbpm_dos(out["corr_mean"], rescale)
        if keep is not None:
            keep.append(out)
        return out

    for i in range(args.warmup):
        t = time.perf_counter()
        one_step(i, None)
        log(f"bench: warmup {i} {time.perf_counter() - t:.2f} s")

    kept = []
    tbpm.tbpm_ctx_set_profiling(ctx.handle, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        one_step(i, kept)
        log(f"bench: step {i} done at {time.perf_counter() - t0:.2f} s")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    tbpm.tbpm_ctx_set_profiling(ctx.handle, False)

    mid_ms, mid_n = tbpm.tbpm_ctx_kernel_time(ctx.handle, 1)
    first_ms, first_n = tbpm.tbpm_ctx_kernel_time(ctx.handle, 0)
    last_ms, last_n = tbpm.tbpm_ctx_kernel_time(ctx.handle, 2)
    terms = len(tbpm.tbpm_coefficients(np.pi)) - 1
    if args.route in ("ac", "dp"):
        # products with H: the Fermi series of two vectors, then both vectors' time steps
        work = lat.nnz * (2 * (fermi_terms - 1) + 2 * terms * nt) * args.steps
    elif args.route in ("moments", "sites"):
        # products with H actually applied: ceil(N/2) per vector
        work = lat.nnz * ((num_moments + 1) // 2) * R * args.steps
    else:
        work = lat.nnz * terms * nt * R * args.steps
    value = work / el
    alg_bytes, h_bytes, terms_per_launch = algorithmic_bytes_per_launch(info, lat.n, B, w["dtype"],
                                                                        clenshaw and args.route != "moments"
                                                                        and args.route != "sites")
    if args.route in ("moments", "sites"):
        # single product: H, a gathered read of p_m, read and write of p_m-1 -> p_m+1 (3 accesses);
        # fused pair (patch format, one vector): H once, reads of p_m, p_m-1, writes of p_m+1, p_m+2
        sv = 16 if w["dtype"] == "c128" else 8
        if info["format"] == 3 and B == 1:
            alg_bytes, terms_per_launch = h_bytes + 4 * sv * lat.n * B, 2
        else:
            alg_bytes, terms_per_launch = h_bytes + 3 * sv * lat.n * B, 1
    mid_avg_s = mid_ms / max(mid_n, 1) / 1e3
    achieved = alg_bytes / mid_avg_s / 1e9 if mid_n else None
    if args.route == "sites" and info["format"] == 3:
        # light cone: each product touches only the patches the sites' states have
        # reached, so bytes per launch vary and the full-matrix figure does not apply
        achieved = None
    kernel_tag = ("cl_" if clenshaw else "") + ("mid_pair" if terms_per_launch == 2 else "mid_term")
    if args.route in ("moments", "sites"):
        kernel_tag = "moment_pair" if terms_per_launch == 2 else "moment_term"
    # the counter summaries were taken with the default matrix layout and block width
    # (and every row of H per launch, which the light cone of --route sites skips)
    default_layout = (args.format == "auto" and not args.large_patches and not args.no_value_table
                      and args.route != "sites")
    series_name = "clenshaw" if clenshaw and args.route not in ("moments", "sites") else "forward"
    traffic = read_traffic(kernel_tag, args.workload, series_name) if default_layout else None
    # the per-step figure of the forward recurrence: (M-1) products, each streaming H once,
    # and (5M-6) vector accesses of s_x n B bytes (3 on the first product, 5 on each later
    # one, one psi0 read for the correlation sums), per block of B vectors
    sv = 16 if w["dtype"] == "c128" else 8
    h_step = (info["ell_w"] * lat.n * (sv + 4) if info["format"] in (1, 3)
              else lat.nnz * (sv + 4) + (lat.n + 1) * (8 if lat.nnz >= 2 ** 31 - 1 else 4))
    step_bytes = terms * h_step + (5 * (terms + 1) - 6) * sv * lat.n * B
    blocks_per_bench_step = max(1, R // B)
    step_rate = (step_bytes * nt * blocks_per_bench_step * args.steps / el / 1e9
                 if args.route == "propagate" else None)
    norms_dev = max(float(np.abs(o["norms"] - 1).max()) for o in kept) if args.route == "propagate" else None
    if args.route == "wft":
        norms_dev = max(float(np.abs(o["snapshot_norms"] - 1).max()) for o in kept)

    cpu = None
    if args.cpu_seconds > 0:
        log("bench: timing the CPU oracle on a bounded sample")
        if args.route == "moments":
            cpu = cpu_baseline_moments(lat, w, args.cpu_seconds, kept[0]["mu"][0] if kept else None)
        elif args.route == "sites":
            cpu = cpu_baseline_moments(lat, w, args.cpu_seconds, kept[0]["mu"][0] if kept else None,
                                       site=int(kept[0]["sites"][0]) if kept else None)
        elif args.route in ("qe", "wft", "ac", "dp"):
            cpu = cpu_baseline(lat, w, args.cpu_seconds,
                               None if args.route in ("ac", "dp") else (kept[0]["corr"][0] if kept else None))
        else:
            c0 = kept[0]["corr"][0] if kept and kept[0]["corr"].shape[0] >= 1 else None
            cpu = cpu_baseline(lat, w, args.cpu_seconds, c0)
            if args.workload in FULL_LENGTH_CHECK and args.route == "propagate" and not clenshaw:
                log("bench: full-length check on a reduced instance")
                cpu["full_length_vs_oracle"] = full_length_check(ctx, tbpm, args.workload, dict(WORKLOADS[args.workload]))

    line = {
        "metric": "Hamiltonian-nnz*Chebyshev-terms/s",
        "route": args.route,
        "value": value,
        "unit": "nnz*terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if w["dtype"] == "c128" else "f32 (f64 update and sums)",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": w["text"], "orbitals": lat.n, "nnz": lat.nnz,
                   "time_steps": nt, "vectors_per_step": R, "block": B, "chebyshev_terms_per_step": terms,
                   "format": fmt_name,
                   **({"series": "clenshaw",
                       "variant": "formulation variant: the same truncated series by Clenshaw's backward "
                                  "recurrence (no accumulator vector); the headline line uses the paper's "
                                  "forward recurrence"} if clenshaw and args.route not in ("moments", "sites")
                      else {"series": "forward"} if args.route not in ("moments", "sites") else {}),
                   **({"qe_energies": qe_energies} if args.route == "qe" else {}),
                   **({"wft_snapshot_steps": wft_steps} if args.route == "wft" else {}),
                   **({"ldos_sites_per_step": n_sites} if args.route == "sites" else {}),
                   **({"kT_eV": args.kT, "mu_eV": args.mu, "fermi_terms": fermi_terms,
                       "operator": "current J_x (sigma_xx)" if args.route == "ac" else "density rho_q, q = 16 x 2pi/L_a",
                       "result_sample": [float(np.real(x)) for x in kept[0]["result"][::6]] if kept else None}
                      if args.route in ("ac", "dp") else {}),
                   **({"chebyshev_moments": num_moments,
                                           "products_with_H_per_vector": (num_moments + 1) // 2,
                                           "propagation_equivalent_value":
                                               lat.nnz * terms * nt * R * args.steps / el}
                                          if args.route in ("moments", "sites") else {})},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                     "traffic": traffic,
                     "kernel": ("moment pair (two fused SpMV + recurrence + <p|p>, <p|p'> partial sums per "
                                "pass over H)" if args.route in ("moments", "sites") and terms_per_launch == 2 else
                                "moment term (fused SpMV + in-place recurrence + <p_m|p_m>, <p_m|p_m+1> "
                                "partial sums)" if args.route in ("moments", "sites") else
                                "middle Clenshaw pair (two fused SpMV of the backward Chebyshev recurrence, "
                                "coefficients folded in, per pass over H)" if terms_per_launch == 2 and clenshaw else
                                "middle Chebyshev term pair (two fused SpMV + recurrence + coefficient updates "
                                "per pass over H)" if terms_per_launch == 2 else
                                "middle Clenshaw term (fused SpMV of the backward Chebyshev recurrence with its "
                                "coefficient)" if clenshaw else
                                "middle Chebyshev term (fused SpMV + recurrence + coefficient update)"),
                     **({"note": "light cone of site-localised states: each product processes only the "
                                 "patches within reach of the sites; value counts full-matrix products"}
                        if args.route == "sites" and info["format"] == 3 else {}),
                     "terms_per_launch": terms_per_launch,
                     "bytes_model": bytes_model_text(info, B, terms_per_launch, clenshaw, args.route),
                     "algorithmic_bytes_per_launch": alg_bytes, "h_bytes_per_launch": h_bytes,
                     "counted_GBps": (traffic / mid_avg_s / 1e9) if (traffic and mid_n) else None,
                     # the per-step figure of the plain format (single terms on slot-major ELL,
                     # 4-byte columns, every value) over the measured step time: an equivalent
                     # rate, above the peak when the stored format moves fewer bytes per step
                     "forward_recurrence_bytes_per_step": step_bytes if args.route == "propagate" else None,
                     "forward_recurrence_step_equiv_GBps": step_rate,
                     "forward_recurrence_step_equiv_frac": (step_rate / HBM_PEAK_GBS) if step_rate else None,
                     "avg_launch_us": mid_avg_s * 1e6, "launches_timed": mid_n,
                     # with Clenshaw the "first" group is the first two products (the first
                     # pair and, when M - 5 is odd, the single product after it)
                     "first_term_avg_us": first_ms / max(first_n, 1) * 1e3,
                     "last_term_avg_us": last_ms / max(last_n, 1) * 1e3},
        "cpu_baseline": cpu,
        "max_norm_drift": norms_dev,
    }
    if ops is not None:
        tbpm.tbpm_ham_destroy(ops[0])
        if args.route == "dp":
            tbpm.tbpm_ham_destroy(ops[1])
    tbpm.tbpm_ham_destroy(ham)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
