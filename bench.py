#!/usr/bin/env python
"""Benchmark of the GKBA collision integral I(t) on one MI355X.

Workload: N = 100 basis functions, T = 1000 past times, dt = 0.05, seeded
synthetic inputs (dense real v of 10^8 entries with the {ijkl, jilk, klij,
lkji} permutation symmetry, Hermitian h, smooth rho history).  One step = one
full I(t) evaluation through the C ABI: propagators, GKBA two-time functions,
2 T second-Born self-energies (48 T N^5 = 4.8e14 algorithmic flops) and the
float64 sum over past times, with all inputs resident in HBM.

Prints one JSON line.  `value` is steps/s of the bulk precision given by
--prec (default: the split-float16 path); the float64 and float32 paths are
timed beside it for the "vs FP64" comparison.  The roofline object refers to
the dominant contraction kernel, timed with HIP events on the launch stream
over the timed region.  The CPU baseline is the FP64 oracle on a bounded
sample of past times, scaled to a full step.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GKBA collision-integral steps/s + MFMA TFLOP/s (N=100,T=1000) vs FP64, at rel err"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "fp16x3": 2516.0}   # MI355X dense matrix peaks
STAGES = ["R1", "R2", "R3", "R4", "layout", "gkba", "pack+reduce", "collision"]
# algorithmic real flops per slice (one self-energy) and stage: complex x real = 4, complex x complex = 8
STAGE_FLOPS_PER_N5 = {"R1": 4, "R2": 8, "R3": 8, "R4": 4}
KERNEL_SOURCES = ["paper_1905_01180_amd/csrc/gemm.hpp", "paper_1905_01180_amd/csrc/stream_gemm.hpp",
                  "paper_1905_01180_amd/csrc/chain.hpp", "paper_1905_01180_amd/csrc/sandwich.hpp",
                  "paper_1905_01180_amd/csrc/r4.hpp"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def rel_f(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:  # pragma: no cover
        pass
    return "unknown"


def cpu_baseline(sys_, nsample: int):
    """FP64 oracle on `nsample` past times, scaled to one full step (T past times).
    `cores` is the number of BLAS threads the oracle's products ran on."""
    from oracle import sb2_oracle as o
    try:
        from threadpoolctl import threadpool_info
        cores = max(int(i.get("num_threads", 1)) for i in threadpool_info()) if threadpool_info() else os.cpu_count()
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    t_len, n = sys_.t, sys_.n
    ks = [t_len - 1 - i * max(1, t_len // max(nsample, 1)) for i in range(nsample)]
    w = o.exchange_combined(sys_.v)
    zero = np.zeros((n, n), np.complex128)
    t0 = time.perf_counter()
    for k in ks:
        u = o.propagator(sys_.h, (t_len - k) * sys_.dt)
        gl, gg, glb, ggb = o.gkba_pair(u, sys_.rho_hist[k], zero)
        o.sigma(sys_.v, gg, glb, w) @ glb - o.sigma(sys_.v, gl, ggb, w) @ ggb
    dt_s = time.perf_counter() - t0
    per_step = dt_s / len(ks) * t_len
    return {"value": 1.0 / per_step, "unit": "steps/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{len(ks)} of {t_len} past times (Sigma^<, Sigma^>, collision term each) at N={n}, "
                      f"{dt_s:.1f} s, scaled by T/{len(ks)} (cost is linear in T)",
            "seconds_per_step": per_step, "cpu": cpu_model(), "threads": int(cores),
            "host_cpus": os.cpu_count()}


def eq4_error(torch, _lib, dev, prec, n, t, nk=3):
    """Error of the path on an interaction with exactly the 8-fold symmetry of
    Eq. 4 (Coulomb-like integrals of real orbitals), where the exchange term is
    not a multiple of the direct one: sampled Sigma^<, Sigma^> against the
    oracle at nk past times (the full I would need the oracle over all T)."""
    from oracle import sb2_oracle as o
    from paper_1905_01180_amd import inputs as gen
    s = gen.make_system(n, t, config_id=2, system_id=1, v_kind="orbitals")
    got, sig = _lib.sb2_collision(torch.from_numpy(s.v).to(dev), torch.from_numpy(s.h).to(dev),
                                  torch.from_numpy(s.rho_hist).to(dev), s.dt, prec, return_sigma=True)
    ks = sorted({0, t // 2, t - 1})[:nk]
    sig = sig[:, torch.as_tensor(ks, device=dev)].cpu().numpy()
    w = o.exchange_combined(s.v)
    zero = np.zeros((n, n), np.complex128)
    worst = 0.0
    for i, k in enumerate(ks):
        u = o.propagator(s.h, (t - k) * s.dt)
        gl, gg, glb, ggb = o.gkba_pair(u, s.rho_hist[k], zero)
        worst = max(worst, rel_f(sig[0, i], o.sigma(s.v, gl, ggb, w)), rel_f(sig[1, i], o.sigma(s.v, gg, glb, w)))
    return {"v": "real-orbital Coulomb-like integrals (8-fold symmetry of Eq. 4)", "sigma_rel_F_max": worst,
            "sigma_ks": ks}


def legs(torch, _lib, gen, dev, prec):
    """Short measurements of the other workloads, reported beside the headline:
    config 1 (N=50, T=500, float64) against its stored oracle values, config 3
    (N=64, T=256: forward and hand-written adjoint, float64), config 4 (32
    systems, N 24..96, T 64..512: one batched call against 32 single calls)
    and the propagation with the carried sum over past times at N = 100."""
    out = {}

    def tsec(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    # config 1: float64 baseline
    s = gen.make_config(1)
    v, h, r = (torch.from_numpy(x).to(dev) for x in (s.v, s.h, s.rho_hist))
    sec = tsec(lambda: _lib.sb2_collision(v, h, r, s.dt, "fp64"), 3)
    c1 = {"workload": "N=50, T=500, float64", "steps_per_s": 1.0 / sec,
          "tflops_algorithmic": 48.0 * s.t * s.n ** 5 / sec / 1e12,
          "frac_fp64_peak": 48.0 * s.t * s.n ** 5 / sec / 1e12 / PEAK_TFLOPS["fp64"]}
    gold = os.path.join(ROOT, "tests", "golden", "oracle_c1.npz")
    if os.path.exists(gold):
        z = np.load(gold)
        c1["I_rel_F"] = rel_f(_lib.sb2_collision(v, h, r, s.dt, "fp64").cpu().numpy(), z["i_ns"])
    out["c1_fp64"] = c1
    del v, h, r
    # config 3: forward + adjoint
    s = gen.make_config(3)
    v, h, r = (torch.from_numpy(x).to(dev) for x in (s.v, s.h, s.rho_hist))
    gi = (1j * h.conj().T).contiguous()          # dL/dI for L = Im tr[h I] in torch's convention
    t_f = tsec(lambda: _lib.sb2_collision(v, h, r, s.dt, "fp64"), 2)
    t_b = tsec(lambda: _lib.sb2_collision_backward(v, h, r, s.dt, gi), 2)
    n5 = float(s.n) ** 5
    out["c3_adjoint_fp64"] = {
        "workload": "N=64, T=256, float64, L = Im tr[h I]", "forward_s": t_f, "backward_s": t_b,
        "backward_over_forward": t_b / t_f,
        # backward: forward chain recomputed (24 N^5 per self-energy) + eight adjoint contractions (48 N^5)
        "backward_tflops_algorithmic": 2 * s.t * 72.0 * n5 / t_b / 1e12,
        "backward_frac_fp64_peak": 2 * s.t * 72.0 * n5 / t_b / 1e12 / PEAK_TFLOPS["fp64"]}
    del v, h, r
    # config 4: batched against single calls (eager)
    systems = gen.make_batch(32, config_id=4)
    data = [tuple(torch.from_numpy(x).to(dev) for x in (q.v, q.h, q.rho_hist)) + (q.dt,) for q in systems]
    t_seq = tsec(lambda: [_lib.sb2_collision(a, b, c, d, prec) for (a, b, c, d) in data], 1)
    t_grp = tsec(lambda: _lib.sb2_collision_batched(data, prec), 1)
    flops = sum(48.0 * q.t * float(q.n) ** 5 for q in systems)
    out["c4_batched"] = {"workload": "32 systems, N ~ U{24..96}, T ~ U{64..512}, " + prec,
                         "batched_s": t_grp, "sequential_s": t_seq, "speedup": t_seq / t_grp,
                         "tflops_algorithmic": flops / t_grp / 1e12}
    del data
    # propagation with the sum over past times carried (float64): steps 2..6 from t_0
    s = gen.make_system(100, 1, config_id=2)
    v, h = torch.from_numpy(s.v).to(dev), torch.from_numpy(s.h).to(dev)
    rho = torch.zeros((8, 100, 100), dtype=torch.complex128, device=dev)
    rho[0].copy_(torch.from_numpy(s.rho_hist[0]))
    pst = torch.zeros((100, 100), dtype=torch.complex128, device=dev)
    mst = torch.zeros((100 ** 4,), dtype=torch.complex128, device=dev)
    _lib.sb2_gkba_propagate_linear(v, h, rho, pst, mst, 0, 2, s.dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _lib.sb2_gkba_propagate_linear(v, h, rho, pst, mst, 2, 5, s.dt)
    torch.cuda.synchronize()
    t_lin = (time.perf_counter() - t0) / 5
    out["propagate_linear_fp64"] = {
        "workload": "GKBA propagation N=100, float64, sum over past times carried (cost per step independent "
                    "of the history)", "ms_per_step": 1e3 * t_lin,
        "tflops_algorithmic": 84.0 * 1e10 / t_lin / 1e12}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", default="fp16x3", choices=["fp64", "fp32", "fp16x3"])
    ap.add_argument("--n", type=int, default=100)
    ap.add_argument("--t", type=int, default=1000)
    ap.add_argument("--no-compare", action="store_true", help="skip timing the other precisions")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-sample", type=int, default=12)
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the short measurements of the other workloads (N=50 FP64, adjoint, batched)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one 256 MiB device copy (calibration point for hardware byte counters)")
    ap.add_argument("--no-error", action="store_true", help="skip the accuracy check against the stored oracle")
    ap.add_argument("--batched", action="store_true",
                    help="measure the 32-system batch (N 24..96, T 64..512): one grouped call vs 32 single calls")
    ap.add_argument("--autotune", action="store_true", help="run sb2_autotune for the workload before timing")
    ap.add_argument("--linear", action="store_true",
                    help="with --propagate: the propagation with the sum over past times carried along (float64)")
    ap.add_argument("--propagate", action="store_true",
                    help="time whole GKBA propagation steps (HF + second-Born collisions) from a history of --t steps")
    ap.add_argument("--vertex", choices=["diagonal", "symmetric"],
                    help="time the special-vertex collision integral (float64) at --n, --t")
    ap.add_argument("--v", choices=["lowrank", "orbitals"], default="lowrank",
                    help="interaction: the workloads' low-rank construction or real-orbital integrals (Eq. 4 symmetry)")
    ap.add_argument("--packed", action="store_true",
                    help="pass v as its 8-fold packed values (sb2_collision_v8; needs --v orbitals)")
    ap.add_argument("--chain", choices=["hubbard", "ohno"],
                    help="the paper's chain propagations of Sec. IV (N_b=10, J=-1, U=1; hubbard: diagonal "
                         "vertex, 5000 steps of 0.01; ohno: symmetric vertex, 2000 steps of 0.025), float64")
    ap.add_argument("--adjoint", action="store_true",
                    help="time the forward and the hand-written adjoint (float64) at --n, --t (default N=64, T=256)")
    ap.add_argument("--small-batch", action="store_true",
                    help="with --batched: 32 small systems (N 8..24, T 16..64) instead of N 24..96, T 64..512")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the method would shard over past times with one all-reduce of I per step; not implemented).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1905_01180_amd import _lib
    from paper_1905_01180_amd import inputs as gen

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    L = _lib.lib()

    if args.batched:
        return batched(args, torch, _lib, gen, dev)
    if args.propagate:
        if args.linear:
            return propagate_linear(args, torch, _lib, gen, dev)
        return propagate(args, torch, _lib, gen, dev)
    if args.vertex:
        return vertex(args, torch, _lib, gen, dev)
    if args.adjoint:
        return adjoint(args, torch, _lib, gen, dev)
    if args.chain:
        return chain(args, torch, _lib, gen, dev)

    cid = 2 if (args.n, args.t) == (100, 1000) else 99
    log(f"generating inputs N={args.n} T={args.t}")
    if args.packed and args.v != "orbitals":
        print("--packed needs an interaction with the 8-fold symmetry: add --v orbitals", file=sys.stderr)
        sys.exit(2)
    s = gen.make_system(args.n, args.t, config_id=cid, v_kind=args.v)
    if args.v != "lowrank":
        args.no_error = True             # the stored oracle values belong to the low-rank interaction
    if args.packed:
        from paper_1905_01180_amd import v8
        vp = torch.from_numpy(v8.pack(s.v)).to(dev)
    v = torch.from_numpy(s.v).to(dev)
    h = torch.from_numpy(s.h).to(dev)
    rho = torch.from_numpy(s.rho_hist).to(dev)
    n5 = float(args.n) ** 5
    flops_step = 48.0 * args.t * n5

    if args.copy_probe:
        src = torch.ones(256 << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def run(prec):
        if args.packed:
            return _lib.sb2_collision_v8(vp, h, rho, s.dt, prec)
        return _lib.sb2_collision(v, h, rho, s.dt, prec)

    tuned = None
    if args.autotune:
        log(f"autotuning {args.prec}")
        tuned = _lib.sb2_autotune(v, h, rho, s.dt, args.prec)
        log(f"tuned: {tuned}")

    def timed(prec, steps, warmup, profile):
        for _ in range(warmup):
            run(prec)
        torch.cuda.synchronize()
        if profile:
            L.sb2_profile_enable(1)
        t0 = time.perf_counter()
        for i in range(steps):
            run(prec)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        stages = None
        if profile:
            import ctypes
            ms = (ctypes.c_double * 8)()
            cnt = (ctypes.c_int * 8)()
            st = L.sb2_profile_read(ms, cnt, 8)
            L.sb2_profile_enable(0)
            if st == 0:
                stages = {STAGES[i]: {"ms_per_step": ms[i] / steps, "launches_per_step": cnt[i] / steps}
                          for i in range(8)}
        return el, stages

    log(f"timing {args.prec}: warmup {args.warmup}, steps {args.steps}")
    el, stages = timed(args.prec, args.steps, args.warmup, True)
    value = args.steps / el
    ms_per_step = 1e3 * el / args.steps

    # dominant contraction kernel
    roof = None
    if stages:
        fused = stages["R3"]["launches_per_step"] == 0 and stages["R2"]["launches_per_step"] > 0
        if fused:                        # the R2 slot times the fused second+third contraction
            stages["R2+R3"] = stages.pop("R2")
            stages.pop("R3")
        flops_n5 = dict(STAGE_FLOPS_PER_N5, **{"R2+R3": 16})
        dom = max((k for k in ("R1", "R2", "R3", "R2+R3", "R4") if k in stages),
                  key=lambda k: stages[k]["ms_per_step"])
        st = stages[dom]
        per_launch_ms = st["ms_per_step"] / max(st["launches_per_step"], 1e-9)
        flops_per_launch = flops_n5[dom] * n5 * 2 * args.t / st["launches_per_step"]
        achieved = flops_per_launch / (per_launch_ms * 1e-3) / 1e12
        peak = PEAK_TFLOPS[args.prec]
        traffic = None
        tf = os.path.join(ROOT, "profiles", f"traffic_{dom.replace('+', '')}_{args.prec}_n{args.n}.json")
        if os.path.exists(tf):
            with open(tf) as fh:
                tj = json.load(fh)
            if tj.get("kernel_hash") == kernel_hash():
                traffic = tj.get("bytes_per_launch")
        roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": traffic, "kernel": dom, "launch_ms": per_launch_ms,
                "flops_per_launch": flops_per_launch,
                "traffic_source": (os.path.relpath(tf, ROOT) + ": rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE of a "
                                   "separate run, calibrated by a device copy; valid for the kernel sources' hash")
                if traffic is not None else "no counter run for the current kernel sources"}
        if args.prec == "fp16x3":
            roof["note"] = ("algorithmic flops vs the dense fp16 peak; each real product costs three fp16 "
                            "MFMAs, so the split method's ceiling is frac = 1/3")

    # accuracy against the stored FP64 oracle (written by tests/golden/make_golden.py)
    err = None
    gold = os.path.join(ROOT, "tests", "golden", f"oracle_c{cid}.npz")
    if os.path.exists(gold) and not args.no_error:
        z = np.load(gold)
        got, sig = _lib.sb2_collision(v, h, rho, s.dt, args.prec, return_sigma=True)
        got, sig = got.cpu().numpy(), sig.cpu().numpy()
        ks = z["sigma_ks"]
        err = {"I_rel_F": rel_f(got, z["i_ns"]),
               "I_rel_maxabs": float(np.abs(got - z["i_ns"]).max() / np.abs(z["i_ns"]).max()),
               "sigma_rel_F_max": max(max(rel_f(sig[0, k], z["sigma_less"][i]),
                                          rel_f(sig[1, k], z["sigma_great"][i])) for i, k in enumerate(ks)),
               "sigma_ks": [int(k) for k in ks],
               "kappa_I": float(z["term_norms"].sum() / np.linalg.norm(z["i_ns"]))}
        del sig
        if (args.n, args.t) == (100, 1000):
            log("error on a real-orbital interaction (Eq. 4 symmetry)")
            err["eq4_interaction"] = eq4_error(torch, _lib, dev, args.prec, args.n, args.t)

    compare = {}
    if not args.no_compare:
        for p in ("fp64", "fp32", "fp16x3"):
            if p == args.prec:
                compare[p] = value
                continue
            log(f"timing {p} for comparison")
            e2, _ = timed(p, 1, 1, False)
            compare[p] = 1.0 / e2

    other = None
    if not args.no_legs and (args.n, args.t) == (100, 1000):
        log("other workloads: N=50 FP64, adjoint N=64 T=256, 32-system batch, carried-sum propagation N=100")
        other = legs(torch, _lib, gen, dev, args.prec)

    cpu = None
    if not args.no_cpu:
        log("timing the CPU oracle sample")
        cpu = cpu_baseline(s, args.cpu_sample)

    out = {
        "metric": METRIC, "value": value, "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.prec, "data": "synthetic",
        "config": {"workload": f"GKBA collision integral, N={args.n} basis, T={args.t} past times, dt={s.dt}",
                   "N": args.n, "T": args.t, "prec": args.prec,
                   **({"interaction": args.v} if args.v != "lowrank" else {}),
                   **({"v_format": "8-fold packed"} if args.packed else {})},
        "tflops_algorithmic": flops_step * value / 1e12,
        "roofline": roof, "cpu_baseline": cpu, "rel_err": err, "steps_per_s_by_prec": compare or None,
        "stages": stages, "kernel_hash": kernel_hash(), "tuning": tuned, "other_workloads": other,
    }
    print(json.dumps(out), flush=True)


def batched(args, torch, _lib, gen, dev):
    """32 systems of uneven size: the grouped entry point (eager and replayed
    from a captured HIP graph) against 32 single-system calls (eager and
    captured).  value = systems/s of the graph-replayed grouped call."""
    rng_n, rng_t = ((8, 24), (16, 64)) if args.small_batch else ((24, 96), (64, 512))
    systems = gen.make_batch(32, config_id=5 if args.small_batch else 4, n_range=rng_n, t_range=rng_t)
    data = [tuple(torch.from_numpy(x).to(dev) for x in (s.v, s.h, s.rho_hist)) + (s.dt,) for s in systems]
    flops = sum(48.0 * s.t * float(s.n) ** 5 for s in systems)
    prec = args.prec

    def seq():
        return [_lib.sb2_collision(v, h, r, dt, prec) for (v, h, r, dt) in data]

    def grp():
        return _lib.sb2_collision_batched(data, prec)

    def time_eager(fn, steps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    def capture(fn):
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            fn()                                     # workspace sized outside capture
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            outs = fn()
        return g, outs

    def time_graph(g, steps):
        g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.replay()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    L = _lib.lib()

    def stage_ms(fn):
        import ctypes
        torch.cuda.synchronize()
        L.sb2_profile_enable(1)
        fn()
        torch.cuda.synchronize()
        ms = (ctypes.c_double * 8)()
        cnt = (ctypes.c_int * 8)()
        st = L.sb2_profile_read(ms, cnt, 8)
        L.sb2_profile_enable(0)
        return {STAGES[i]: [round(ms[i], 3), cnt[i]] for i in range(8)} if st == 0 else None

    log(f"batched: 32 systems, {prec}, eager")
    t_seq = time_eager(seq, args.steps)
    t_grp = time_eager(grp, args.steps)
    prof = {"single_calls": stage_ms(seq), "grouped": stage_ms(grp)}
    # parity of the two paths on this workload
    a, b = seq(), grp()
    dev_max = max(float((x - y).abs().max() / y.abs().max()) for x, y in zip(b, a))
    log("batched: graphs")
    g_seq, _ = capture(seq)
    t_seq_g = time_graph(g_seq, args.steps)
    del g_seq
    g_grp, outs = capture(grp)
    t_grp_g = time_graph(g_grp, args.steps)
    replay_equal = all(torch.equal(x, y) for x, y in zip(outs, b))
    out = {
        "metric": "batched GKBA collision integrals: systems/s (32 systems, N %d..%d, T %d..%d)" % (rng_n + rng_t),
        "value": 32.0 / t_grp_g, "unit": "systems/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": 1e3 * t_grp_g, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": prec, "data": "synthetic",
        "config": {"workload": "32 independent systems, N ~ U{%d..%d}, T ~ U{%d..%d}, one I(t) each" % (rng_n + rng_t),
                   "shapes": [[s.n, s.t] for s in systems]},
        "ms": {"single_calls_eager": 1e3 * t_seq, "single_calls_graph": 1e3 * t_seq_g,
               "grouped_eager": 1e3 * t_grp, "grouped_graph": 1e3 * t_grp_g},
        "speedup_grouped_graph_vs_single_eager": t_seq / t_grp_g,
        "speedup_grouped_graph_vs_single_graph": t_seq_g / t_grp_g,
        "tflops_algorithmic": flops / t_grp_g / 1e12,
        "grouped_vs_single_max_rel_diff": dev_max, "graph_replay_bitwise_equal": replay_equal,
        "stage_ms_and_launches": prof,
    }
    print(json.dumps(out), flush=True)


def vertex(args, torch, _lib, gen, dev):
    """Collision integral for a special vertex (Sec. III A / III B), float64:
    the GKBA functions and the sum over past times as in the general path, the
    self-energy by Eq. 14 (diagonal) or Eqs. 16-17 (symmetric).  value = I(t)
    evaluations per second.  The roofline entry covers the self-energy stage:
    for the symmetric basis its exchange and bubble products (16 T N^4 +
    32 T N^3 flops) against the FP64 matrix-core peak."""
    import ctypes
    import numpy as np
    n, t = args.n, args.t
    cid = 2 if (n, t) == (100, 1000) else 99
    log(f"vertex {args.vertex}: N={n} T={t}")
    s = gen.make_system(n, t, config_id=cid)
    g = gen.rng(cid, 0, 9)
    if args.vertex == "diagonal":
        param = torch.from_numpy(g.uniform(0.2, 1.0, n)).to(dev)
    else:
        idx = np.arange(n)
        param = torch.from_numpy(0.5 / np.sqrt(1.0 + (idx[:, None] - idx[None, :]) ** 2.0)).to(dev)
    h = torch.from_numpy(s.h).to(dev)
    rho = torch.from_numpy(s.rho_hist).to(dev)
    run = lambda: _lib.sb2_collision_vertex(args.vertex, param, h, rho, s.dt)
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    L = _lib.lib()
    L.sb2_profile_enable(1)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    ms = (ctypes.c_double * 8)()
    cnt = (ctypes.c_int * 8)()
    st = L.sb2_profile_read(ms, cnt, 8)
    L.sb2_profile_enable(0)
    stages = {"gkba": ms[5] / args.steps, "sigma": ms[6] / args.steps, "collision": ms[7] / args.steps} \
        if st == 0 else None
    n3, n4 = float(n) ** 3, float(n) ** 4
    common = 40.0 * t * n3                     # propagators, X/Y, collision terms (complex MAC = 8 flops)
    sig_flops = 16.0 * t * n4 + 32.0 * t * n3 if args.vertex == "symmetric" else 2.0 * t * n * n * 8.0
    roof = None
    if stages and args.vertex == "symmetric":
        ach = sig_flops / (stages["sigma"] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": ach, "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                "frac": ach / PEAK_TFLOPS["fp64"], "traffic": None, "kernel": "self-energy stage (sym. basis)"}
    out = {
        "metric": "special-vertex GKBA collision integral steps/s (N=%d, T=%d, %s basis)" % (n, t, args.vertex),
        "value": 1.0 / sec, "unit": "steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * sec, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "GKBA collision integral, %s-basis vertex, N=%d, T=%d, dt=%g" % (args.vertex, n, t, s.dt),
                   "N": n, "T": t},
        "tflops_algorithmic": (common + sig_flops) / sec / 1e12, "roofline": roof, "stage_ms": stages,
    }
    print(json.dumps(out), flush=True)


def adjoint(args, torch, _lib, gen, dev):
    """Forward and hand-written adjoint of the collision integral (float64) for
    the scalar L = Im tr[h I] (config 3: N=64, T=256 unless --n/--t are given).
    value = backward passes/s; algorithmic flops of the backward: the forward
    chain recomputed (24 N^5 per self-energy) and the eight adjoint
    contractions (48 N^5 per self-energy), against the FP64 matrix-core peak."""
    n, t = (64, 256) if (args.n, args.t) == (100, 1000) else (args.n, args.t)
    s = gen.make_config(3) if (n, t) == (64, 256) else gen.make_system(n, t, config_id=99)
    v, h, r = (torch.from_numpy(x).to(dev) for x in (s.v, s.h, s.rho_hist))
    gi = (1j * h.conj().T).contiguous()          # dL/dI for L = Im tr[h I] (torch convention)

    def tsec(fn, reps, warm):
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    log(f"adjoint: N={n} T={t}")
    t_f = tsec(lambda: _lib.sb2_collision(v, h, r, s.dt, "fp64"), args.steps, args.warmup)
    t_b = tsec(lambda: _lib.sb2_collision_backward(v, h, r, s.dt, gi), args.steps, args.warmup)
    n5 = float(n) ** 5
    fl_b = 2 * t * 72.0 * n5
    ach = fl_b / t_b / 1e12
    out = {
        "metric": "collision-integral adjoint passes/s (N=%d, T=%d, float64)" % (n, t),
        "value": 1.0 / t_b, "unit": "backward/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * t_b, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "adjoint of the GKBA collision integral, L = Im tr[h I], N=%d, T=%d" % (n, t),
                   "N": n, "T": t},
        "forward_ms": 1e3 * t_f, "backward_over_forward": t_b / t_f,
        "roofline": {"bound": "mfma", "achieved": ach, "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                     "frac": ach / PEAK_TFLOPS["fp64"], "traffic": None, "kernel": "whole backward pass"},
    }
    print(json.dumps(out), flush=True)


# the paper's single-core runtimes of these runs (Table I): loop, contraction (s)
PAPER_CHAIN_S = {"hubbard": (177.0, 164.0), "ohno": (1213.0, 731.0)}


def chain(args, torch, _lib, gen, dev):
    """The chain propagations of Sec. IV on the device: N_b = 10 sites, hopping
    J = -1, on-site U = 1 (Hubbard, diagonal vertex: 5000 steps of 0.01) or
    the Ohno interaction V_ij = U / sqrt(1 + |i - j|^2) (symmetric vertex:
    2000 steps of 0.025), starting with the left half filled (the state a
    strong confinement gives), HF + second-Born collisions, float64.  The
    whole run is one library call; value = time steps per second."""
    n = 10
    vertex, steps, dt = ("diagonal", 5000, 0.01) if args.chain == "hubbard" else ("symmetric", 2000, 0.025)
    h = torch.from_numpy(gen.chain_hopping(n, -1.0)).to(dev)
    par = gen.hubbard_onsite(n, 1.0) if vertex == "diagonal" else gen.ohno_matrix(n, 1.0)
    par = torch.from_numpy(par).to(dev)
    rho = torch.zeros((steps + 1, n, n), dtype=torch.complex128, device=dev)
    u = torch.zeros((steps, n, n), dtype=torch.complex128, device=dev)
    rho[0].copy_(torch.from_numpy(gen.left_half_density(n)))
    log(f"chain {args.chain}: {steps} steps of {dt}")
    # warm-up: a short run on scratch copies (library load, kernel code objects)
    r2, u2 = rho[:11].clone(), u[:10].clone()
    _lib.sb2_gkba_propagate_vertex(vertex, par, h, r2, u2, 0, 10, dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _lib.sb2_gkba_propagate_vertex(vertex, par, h, rho, u, 0, steps, dt)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    occ = torch.diagonal(rho, dim1=1, dim2=2).real.cpu().numpy()
    tr = occ.sum(axis=1)
    every = steps // 10
    loop_s, contr_s = PAPER_CHAIN_S[args.chain]
    out = {
        "metric": "GKBA chain propagation steps/s (Sec. IV, N_b=10, %s vertex, %d steps of %g)" % (vertex, steps, dt),
        "value": steps / wall, "unit": "steps/s", "n_gpus": 1, "steps": steps, "warmup": 1,
        "ms_per_step": 1e3 * wall / steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "%s chain, N_b=10, J=-1, U=1, left half filled at t=0, HF + 2B, %d x %g" %
                               (args.chain, steps, dt), "N": n, "steps": steps, "dt": dt},
        "wall_s": wall, "trace_drift": float(np.abs(tr - tr[0]).max() / tr[0]),
        "left_half_occupation": {f"t={m * dt:g}": float(occ[m, : n // 2].sum()) for m in range(0, steps + 1, every)},
        "site_occupation_final": [float(x) for x in occ[-1]],
        "paper_single_core_s": {"loop": loop_s, "contraction": contr_s,
                                "hardware": "Intel Core i5-4460, 1 core (context, other machine)"},
    }
    print(json.dumps(out), flush=True)


def propagate_linear(args, torch, _lib, gen, dev):
    """Propagation with the sum over past times carried along
    (sb2_gkba_propagate_linear, float64): --warmup then --steps steps from
    t_0 (the cost of a step does not depend on the history length), and, for
    comparison in the same run, --steps steps of the growing-history
    propagation (sb2_gkba_propagate, float64) at history --t.
    value = carried-sum propagation steps/s."""
    import numpy as np
    n, n0 = args.n, args.t
    cid = 2 if (n, n0) == (100, 1000) else 99
    s = gen.make_system(n, n0 + 1, config_id=cid)
    v = torch.from_numpy(s.v).to(dev)
    h = torch.from_numpy(s.h).to(dev)
    stream = torch.cuda.current_stream(dev)

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    # carried sum from t_0
    total = args.warmup + args.steps
    log(f"propagate --linear: N={n}, {total} steps from t_0, float64")
    rho = torch.zeros((total + 1, n, n), dtype=torch.complex128, device=dev)
    rho[0].copy_(torch.from_numpy(s.rho_hist[0]))
    p = torch.zeros((n, n), dtype=torch.complex128, device=dev)
    m = torch.zeros((n ** 4,), dtype=torch.complex128, device=dev)
    if args.warmup:
        _lib.sb2_gkba_propagate_linear(v, h, rho, p, m, 0, args.warmup, s.dt)
    sec = timed(lambda: _lib.sb2_gkba_propagate_linear(v, h, rho, p, m, args.warmup, args.steps, s.dt)) / args.steps
    flops = 84.0 * float(n) ** 5
    tr = torch.diagonal(rho, dim1=1, dim2=2).sum(-1)
    # growing-history steps at history n0 (synthetic state as in --propagate)
    log(f"growing-history propagation at history {n0} for comparison")
    rg = torch.zeros((n0 + args.steps + 1, n, n), dtype=torch.complex128, device=dev)
    rg[: n0 + 1].copy_(torch.from_numpy(s.rho_hist))
    u = torch.zeros((n0 + args.steps, n, n), dtype=torch.complex128, device=dev)
    if n0 > 0:
        u[:n0].copy_(torch.from_numpy(gen.unitary_path(s.h, s.dt * np.arange(n0, 0, -1))))
    sec_g = timed(lambda: _lib.sb2_gkba_propagate(v, h, rg, u, n0, args.steps, s.dt, "fp64")) / args.steps
    out = {
        "metric": "GKBA propagation steps/s (N=%d, HF + second-Born collisions, sum over past times carried)" % n,
        "value": 1.0 / sec, "unit": "steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * sec, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "GKBA propagation, N=%d basis, steps %d..%d from t_0, dt=%g" % (
            n, args.warmup, total, s.dt), "N": n, "prec": "fp64"},
        "flops_per_step": flops, "tflops_algorithmic": flops / sec / 1e12,
        "trace_drift": float((tr - tr[0]).abs().max() / tr[0].abs()),
        "growing_history": {"history": n0, "ms_per_step": 1e3 * sec_g,
                            "flops_per_step": 48.0 * n0 * float(n) ** 5, "speedup": sec_g / sec},
    }
    print(json.dumps(out), flush=True)


def propagate(args, torch, _lib, gen, dev):
    """Whole propagation steps of Sec. II (Sigma_HF, step exponential, collision
    integral over all past times, density step, propagator history) from step
    n0 = --t: the starting state is synthetic (the density history of the
    headline workload, and exp(-i h (t_n0 - t_k)) standing in for the
    propagators of an earlier run).  value = propagation steps/s."""
    import numpy as np
    n, n0, prec = args.n, args.t, args.prec
    cid = 2 if (n, n0) == (100, 1000) else 99
    log(f"propagate: N={n}, history {n0}, {prec}")
    s = gen.make_system(n, n0 + 1, config_id=cid)
    total = n0 + args.warmup + args.steps
    v = torch.from_numpy(s.v).to(dev)
    h = torch.from_numpy(s.h).to(dev)
    rho = torch.zeros((total + 1, n, n), dtype=torch.complex128, device=dev)
    rho[: n0 + 1].copy_(torch.from_numpy(s.rho_hist))
    u = torch.zeros((total, n, n), dtype=torch.complex128, device=dev)
    if n0 > 0:
        u[:n0].copy_(torch.from_numpy(gen.unitary_path(s.h, s.dt * np.arange(n0, 0, -1))))
    ih = torch.zeros((total, n, n), dtype=torch.complex128, device=dev)
    if args.warmup:
        _lib.sb2_gkba_propagate(v, h, rho, u, n0, args.warmup, s.dt, prec, i_hist=ih)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n1 = n0 + args.warmup
    e0.record(stream)
    _lib.sb2_gkba_propagate(v, h, rho, u, n1, args.steps, s.dt, prec, i_hist=ih)
    e1.record(stream)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / args.steps
    flops = sum(48.0 * m * float(n) ** 5 for m in range(n1, n1 + args.steps)) / args.steps
    tr = torch.diagonal(rho[: total + 1], dim1=1, dim2=2).sum(-1)
    out = {
        "metric": "GKBA propagation steps/s (N=%d, history %d, HF + second-Born collisions)" % (n, n0),
        "value": 1.0 / sec, "unit": "steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * sec, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": prec, "data": "synthetic",
        "config": {"workload": "GKBA propagation, N=%d basis, steps %d..%d, dt=%g" % (n, n1, n1 + args.steps, s.dt),
                   "N": n, "n0": n0, "prec": prec},
        "tflops_algorithmic": flops / sec / 1e12,
        "trace_drift": float((tr[n0:] - tr[n0]).abs().max() / tr[n0].abs()),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
