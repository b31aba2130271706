#!/usr/bin/env python3
"""Benchmark of the MI355X MLFMA matvec (one GPU).

A step is one full matvec phi = A q through the C ABI: gather, near-field
P2P, C2M, M2M up the tree, M2L on every level, L2L down the tree, L2O and
the scatter back to the caller's order.  Inputs are resident in HBM before
the timed region; setup (tree, FP64 operator precompute, uploads) is timed
separately.  Prints ONE JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                  [--nrhs R] [--bf16x3] [--no-cpu-baseline] [--no-extras]

The default workload is the 262,144-point sphere of diameter 16 wavelengths,
leaf 0.25 wavelength, 3 digits, one right-hand side.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3        # FP32 vector and FP32 matrix
PEAK_BF16_TFLOPS = 2500.0       # dense BF16 MFMA

# bound of each kernel as implemented
BOUND = {"gather": "hbm", "p2p": "alu", "c2m": "alu", "interp_s1": "mfma",
         "interp_s2": "mfma", "interp_s3": "mfma", "m2l": "alu", "anterp_s1": "mfma",
         "anterp_s2": "mfma", "anterp_s3": "mfma", "l2o": "alu", "interp": "mfma",
         "anterp": "mfma"}


# shift of the second-kind system solved by the GMRES leg: of the order of
# the operator's spectral radius at these point densities (about 330 points
# per square wavelength on the spheres)
GMRES_SHIFT = 1000j


def algorithmic_work(tinfo, levels, R, onepass_up=None, onepass_down=None):
    """Algorithmic bytes and flops of each kernel for one step with R
    right-hand sides (complex64 = 8 bytes; a complex multiply-add = 8 flops;
    a complex-by-real multiply-add = 4 flops; sin, cos and rsqrt count as one
    flop each).  Each quantity is the minimum the method must move or
    compute, not what a kernel happens to do.  onepass_up / onepass_down
    list, per level, whether the pair (l, l+1) runs the one-pass kernel
    (its work is then booked on "interp" / "anterp", else on the three
    staged kernels)."""
    N = tinfo["n_points"]
    nl = tinfo["n_levels"]
    lv = {d["level"]: d for d in levels}
    w = {k: {"bytes": 0.0, "flops": 0.0} for k in BOUND}
    w["gather"]["bytes"] = N * (16.0 * R + 4)
    # per pair: 6 subtractions, 5 for r^2, rsqrt, r, k r, sin, cos, 2 scalings
    # (17) plus a complex multiply-add per right-hand side
    w["p2p"]["flops"] = tinfo["n_p2p_pairs"] * (17.0 + 8.0 * R)
    w["p2p"]["bytes"] = N * (16.0 + 16.0 * R)
    if nl >= 3:
        Kl = lv[nl]["K"]
        # per (point, sample): phase (5), sin + cos (2), complex MAC per RHS
        w["c2m"]["flops"] = N * Kl * (7.0 + 8.0 * R)
        w["c2m"]["bytes"] = N * (16.0 + 8.0 * R) + lv[nl]["nbox"] * R * Kl * 8.0
        w["l2o"]["flops"] = N * Kl * (7.0 + 2.0 + 8.0 * R)
        w["l2o"]["bytes"] = N * (16.0 + 24.0 * R) + lv[nl]["nbox"] * R * Kl * 8.0
        for l in range(3, nl + 1):
            d = lv[l]
            w["m2l"]["bytes"] += 8.0 * R * d["nbox"] * d["K"] * 2 + 8.0 * d["n_types"] * d["K"] \
                + 6.0 * d["n_far"]
            w["m2l"]["flops"] += 8.0 * R * d["n_far"] * d["K"]
        for l in range(3, nl):
            p, c = lv[l], lv[l + 1]
            M = 2 * c["L"] + 1
            Bc, Bp = c["nbox"] * R, p["nbox"] * R
            f1 = 4.0 * Bc * c["ntheta"] * c["nphi"] * M
            f2 = 4.0 * Bc * M * p["ntheta"] * c["ntheta"]
            f3 = 4.0 * Bc * p["ntheta"] * M * p["nphi"] + 8.0 * Bc * p["K"]
            g1 = 4.0 * Bc * p["ntheta"] * p["nphi"] * M + 8.0 * Bc * p["K"]
            g2 = 4.0 * Bc * M * c["ntheta"] * p["ntheta"]
            g3 = 4.0 * Bc * c["ntheta"] * M * c["nphi"]
            up = bool(onepass_up and onepass_up[l - 1] >= 1)
            dn = bool(onepass_down and onepass_down[l - 1] >= 1)
            if up:
                w["interp"]["flops"] += f1 + f2 + f3
                w["interp"]["bytes"] += 8.0 * (Bc * c["K"] + Bp * p["K"])
            if dn:
                w["anterp"]["flops"] += g1 + g2 + g3
                w["anterp"]["bytes"] += 8.0 * (Bp * p["K"] + 2 * Bc * c["K"])
            if not up:
                w["interp_s1"]["flops"] += f1
                w["interp_s1"]["bytes"] += 8.0 * Bc * (c["K"] + c["ntheta"] * M)
                w["interp_s2"]["flops"] += f2
                w["interp_s2"]["bytes"] += 8.0 * Bc * M * (c["ntheta"] + p["ntheta"])
                w["interp_s3"]["flops"] += f3
                w["interp_s3"]["bytes"] += 8.0 * (Bc * p["ntheta"] * M + Bp * p["K"])
            if not dn:
                w["anterp_s1"]["flops"] += g1
                w["anterp_s1"]["bytes"] += 8.0 * (Bc * p["ntheta"] * M + Bp * p["K"])
                w["anterp_s2"]["flops"] += g2
                w["anterp_s2"]["bytes"] += 8.0 * Bc * M * (c["ntheta"] + p["ntheta"])
                w["anterp_s3"]["flops"] += g3
                w["anterp_s3"]["bytes"] += 8.0 * Bc * (c["ntheta"] * M + 2 * c["K"])
    return w


# source file of each kernel: a recorded traffic measurement is used only
# while this file is unchanged
KERNEL_SOURCE = {"m2l": "m2l.hip", "interp": "fused.hip", "anterp": "fused.hip",
                 "p2p": "kernels.hip", "c2m": "kernels.hip", "l2o": "kernels.hip",
                 "gather": "kernels.hip"}
for _k in ("interp_s1", "interp_s2", "interp_s3", "anterp_s1", "anterp_s2", "anterp_s3"):
    KERNEL_SOURCE[_k] = "interp.hip"


def recorded_traffic(kernel, workload, nrhs, forms=None):
    """HBM bytes per launch of `kernel` on `workload`, from the committed
    rocprofv3 counter summary profiles/<kernel>_<workload>_hbm_traffic.txt
    (FETCH_SIZE and WRITE_SIZE runs, scaled by the copy-kernel factors), or
    None when there is none, the kernel source changed since, or the summary
    names the per-level forms it was taken with and `forms` differs."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "%s_%s_hbm_traffic.txt" % (kernel, workload))
    src = KERNEL_SOURCE.get(kernel)
    if not src or not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    with open(os.path.join(ROOT, "paper_2006_15367_amd", "csrc", src), "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()
    if kv.get("source_sha256") != digest or int(kv.get("nrhs", -1)) != nrhs:
        return None
    if "forms" in kv and forms is not None and json.loads(kv["forms"]) != list(forms):
        return None
    return float(kv["traffic_bytes_per_launch"])


def roofline(kernel, work, ms_per_step, launches_per_step, bf16x3):
    bound = BOUND[kernel]
    sec = ms_per_step * 1e-3
    if bound == "hbm":
        achieved = work["bytes"] / sec / 1e9
        peak, unit = PEAK_HBM_GBS, "GB/s"
    else:
        achieved = work["flops"] / sec / 1e12
        peak, unit = PEAK_FP32_TFLOPS, "TFLOP/s"
        if bound == "mfma" and bf16x3:
            peak = PEAK_BF16_TFLOPS
    return {"bound": bound, "kernel": kernel, "achieved": round(achieved, 3), "peak": peak,
            "unit": unit, "frac": round(achieved / peak, 4), "traffic": None,
            "launches_per_step": launches_per_step,
            "avg_launch_us": round(1e3 * ms_per_step / max(1, launches_per_step), 3),
            "ms_per_step": round(ms_per_step, 4)}


# the method's phases (Sec. 2 five-stage list plus the near field) and the
# kernels that run them; a phase's bound is that of its kernels
PHASES = {"gather": ["gather"], "p2p": ["p2p"], "c2m": ["c2m"],
          "m2m": ["interp_s1", "interp_s2", "interp_s3", "interp"],
          "m2l": ["m2l"],
          "l2l": ["anterp_s1", "anterp_s2", "anterp_s3", "anterp"],
          "l2o": ["l2o"]}
PHASE_BOUND = {"gather": "hbm", "p2p": "alu", "c2m": "alu", "m2m": "mfma", "m2l": "alu",
               "l2l": "mfma", "l2o": "alu"}


def phase_rooflines(work, per_kernel_ms, bf16x3):
    """Per phase: algorithmic work, time alone (ms per step, kernels on one
    stream), achieved rate against the peak of its bound, and the floor
    time max(bytes / HBM peak, flops / compute peak).  Also the sum of the
    floors (the whole matvec's roofline time)."""
    out = {}
    floor_total = 0.0
    for ph, ks in PHASES.items():
        fl = sum(work[k]["flops"] for k in ks)
        by = sum(work[k]["bytes"] for k in ks)
        ms = sum(per_kernel_ms.get(k, 0.0) for k in ks)
        bound = PHASE_BOUND[ph]
        cpeak = PEAK_BF16_TFLOPS if (bound == "mfma" and bf16x3) else PEAK_FP32_TFLOPS
        floor_ms = max(by / (PEAK_HBM_GBS * 1e9), fl / (cpeak * 1e12)) * 1e3
        floor_total += floor_ms
        if ms <= 0.0:
            continue
        if bound == "hbm":
            ach, peak, unit = by / (ms * 1e-3) / 1e9, PEAK_HBM_GBS, "GB/s"
        else:
            ach, peak, unit = fl / (ms * 1e-3) / 1e12, cpeak, "TFLOP/s"
        out[ph] = {"bound": bound, "achieved": round(ach, 3), "peak": peak, "unit": unit,
                   "frac": round(ach / peak, 4), "ms_alone": round(ms, 4),
                   "floor_ms": round(floor_ms, 5),
                   "hbm_GBs": round(by / (ms * 1e-3) / 1e9, 1)}
    return out, floor_total


def dense_baseline(xyz, q, ntgt=2048, seed=11):
    """The plain O(N^2) FP64 sum (C, OpenMP on the host cores) on a bounded
    sample of targets: pairs per second and the extrapolated full time."""
    from oracle import dense
    from paper_2006_15367_amd import workloads as W
    rng = np.random.default_rng(seed)
    idx = rng.choice(xyz.shape[0], min(ntgt, xyz.shape[0]), replace=False)
    R = 1 if q.ndim == 1 else q.shape[1]
    dense.potential(xyz[:64], q[:64], W.K_WAVENUMBER)   # load the library
    t0 = time.perf_counter()
    dense.potential(xyz, q, W.K_WAVENUMBER, tgt=xyz[idx])
    dt = time.perf_counter() - t0
    pairs = float(idx.size) * xyz.shape[0] * R
    return {"pairs_per_s": round(pairs / dt, 1), "targets": int(idx.size),
            "seconds": round(dt, 3),
            "full_matvec_s_extrapolated": round(dt * xyz.shape[0] / idx.size, 2)}


def cpu_baseline(xyz, q, phi_gpu, repeats=3):
    """The FP64 oracle MLFMA, untuned, timed on the host cores: the median
    of `repeats` full matvecs of the same workload (setup excluded), plus
    the plain dense sum on 2,048 sampled targets."""
    from oracle import dense
    from oracle import mlfma as M
    from paper_2006_15367_amd import workloads as W
    tree = M.Tree(xyz, W.LEAF_SIZE)
    ops = M.Operators(tree, W.K_WAVENUMBER, W.DIGITS)
    times = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        phi = M.matvec(tree, ops, q)
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    R = 1 if q.ndim == 1 else q.shape[1]
    err = float(np.linalg.norm(phi_gpu - phi) / np.linalg.norm(phi))
    rng = np.random.default_rng(7)
    idx = rng.choice(xyz.shape[0], min(1024, xyz.shape[0]), replace=False)
    ref = dense.potential(xyz, q, W.K_WAVENUMBER, tgt=xyz[idx])
    err_dense = float(np.linalg.norm(phi_gpu[idx] - ref) / np.linalg.norm(ref))
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    import platform
    cpu_model = platform.processor() or ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": round(xyz.shape[0] * R / dt, 1), "unit": "points/s", "cores": cores,
            "kind": "oracle", "seconds": round(dt, 3),
            "seconds_each": [round(t, 3) for t in times], "cpu": cpu_model,
            "sample": "median of %d full FP64 oracle MLFMA matvecs of the same workload "
                      "(numpy + C near field), setup excluded" % repeats,
            "dense": dense_baseline(xyz, q),
            "gpu_rel_l2_vs_oracle_mlfma": err, "gpu_rel_l2_vs_dense_1024_targets": err_dense}


def _timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def _dense_check(xyz, q, phi, ntgt=128, ncol=4):
    """rel. L2 of a GPU result against the dense FP64 sum on sampled targets
    (at most ncol right-hand sides)."""
    from oracle import dense
    from paper_2006_15367_amd import workloads as W
    rng = np.random.default_rng(3)
    idx = rng.choice(xyz.shape[0], ntgt, replace=False)
    qq = q if q.ndim == 1 else q[:, :ncol]
    pp = phi[idx] if phi.ndim == 1 else phi[idx, :ncol]
    ref = dense.potential(xyz, np.ascontiguousarray(qq).astype(np.complex128),
                          W.K_WAVENUMBER, tgt=xyz[idx])
    return float(np.linalg.norm(pp - ref) / np.linalg.norm(ref))


def extra_workloads(headline_ms, headline_operator_bytes=None, steps=5, warmup=2):
    """The other benchmark configurations, timed in the same run (inputs
    resident, default schedule): the elongated cloud with its tip cluster,
    64 right-hand sides in FP32 and with BF16x3 interpolation, the volume
    cloud with 16 right-hand sides (matvec, and loss + backward of
    ||phi - phi_target||^2 through the adjoint and field passes), and the
    benchmark sphere and the elongated cloud with sampled translation
    operators (operator memory against the full tables)."""
    import gc
    import torch
    from paper_2006_15367_amd import mlfma as G
    from paper_2006_15367_amd import workloads as W
    from paper_2006_15367_amd.autograd import potential
    out = {}
    r64_fp32 = None
    full_mem = {"sphere262k": headline_operator_bytes}
    for key, name, bf, samp in (("spheroid1m", "spheroid1m", False, False),
                                ("sphere262k_r64", "sphere262k_r64", False, False),
                                ("sphere262k_r64_bf16x3", "sphere262k_r64", True, False),
                                ("cube1m_r16", "cube1m_r16", False, False),
                                ("sphere262k_sampled_operators", "sphere262k", False, True),
                                ("spheroid1m_sampled_operators", "spheroid1m", False, True)):
        try:
            xyz, q = W.make(name)
            R = 1 if q.ndim == 1 else q.shape[1]
            t0 = time.perf_counter()
            tree = G.Tree(xyz, W.LEAF_SIZE)
            ops = G.Operators(tree, W.K_WAVENUMBER, W.DIGITS, max_rhs=R, bf16x3=bf,
                              sampled=samp)
            torch.cuda.synchronize()
            setup = time.perf_counter() - t0
            qd = torch.from_numpy(np.ascontiguousarray(q.astype(np.complex64))).cuda()
            ms = _timed(lambda: ops.matvec(qd), steps, warmup)
            phi = ops.matvec(qd)
            torch.cuda.synchronize()
            e = {"n_points": int(xyz.shape[0]), "nrhs": R, "ms_per_matvec": round(ms, 3),
                 "points_x_rhs_per_s": round(xyz.shape[0] * R / (ms * 1e-3), 1),
                 "setup_s": round(setup, 2), "levels": tree.info()["n_levels"],
                 "rel_l2_vs_dense_128_targets": _dense_check(xyz, q, phi.cpu().numpy())}
            if R > 1:
                e["ms_per_rhs"] = round(ms / R, 4)
            mem = ops.memory()
            e["operator_bytes"] = mem["operator_bytes"]
            if not samp and R == 1:
                full_mem[name] = mem["operator_bytes"]
            if samp:
                e["m2l_variant_per_level"] = ops.variants("m2l")
                if name == "sphere262k":
                    e["slowdown_vs_full_tables_headline"] = round(ms / headline_ms, 3)
                if full_mem.get(name):
                    e["full_table_operator_bytes"] = full_mem[name]
            if name == "sphere262k_r64":
                # same cloud as the headline: batched against single-RHS calls
                e["speedup_per_rhs_vs_single_rhs_headline"] = round(headline_ms * R / ms, 3)
            if key == "sphere262k_r64":
                r64_fp32 = ms
            if key == "sphere262k_r64_bf16x3" and r64_fp32:
                e["speedup_vs_fp32_r64"] = round(r64_fp32 / ms, 3)
            if key == "cube1m_r16":
                tq = torch.from_numpy(W.charges(xyz.shape[0], R, seed=1)).cuda()
                with torch.no_grad():
                    target = ops.matvec(tq)
                xg = torch.from_numpy(xyz).cuda()

                def step():
                    qq = qd.clone().requires_grad_(True)
                    xx = xg.clone().requires_grad_(True)
                    L = (potential(qq, xx, ops) - target).abs().pow(2).sum()
                    L.backward()
                e["loss_backward_ms"] = round(_timed(step, steps, warmup), 3)
                e["loss_backward"] = ("||phi - phi_t||^2, phi_t = A q_t (charges seed 1); "
                                      "grads w.r.t. complex charges and positions")
                del target, xg, tq
            out[key] = e
            del ops, tree, qd, phi
        except Exception as ex:  # keep the headline line whatever happens here
            out[key] = {"error": "%s: %s" % (type(ex).__name__, ex)}
        gc.collect()
        torch.cuda.empty_cache()
    return out


def smooth_phi_count(L):
    """Smallest even phi count >= 2 L + 2 with no prime factor above 7 (the
    uniform grids of the FFT interpolation)."""
    P = 2 * L + 2
    while True:
        m = P
        for r in (2, 3, 5, 7):
            while m % r == 0:
                m //= r
        if m == 1 and P % 2 == 0:
            return P
        P += 1


def fft_ablation(levels, nrhs, dense_phases, reps=20):
    """The FFT interpolation (Sec. 3.2.2, Fig. 3) and its weighted-adjoint
    anterpolation on uniform grids, timed on every level pair of the
    workload with one item per child box and right-hand side, beside the
    dense MFMA maps of the matvec (M2M and L2L phases alone, which also
    shift and aggregate).  Algorithmic bytes: each item's input and output
    grid once."""
    import torch
    from paper_2006_15367_amd import mlfma as G
    lv = {e["level"]: e for e in levels if e["L"] > 0}
    out = {"pairs": [], "grid": "uniform: P phi x P/2 theta samples, P = smallest 7-smooth "
                                "even >= 2L + 2"}
    tot = {False: 0.0, True: 0.0}
    byt = {False: 0.0, True: 0.0}
    for l in sorted(lv):
        if l + 1 not in lv:
            continue
        Lc, Lp = lv[l + 1]["L"], lv[l]["L"]
        Pc, Pp = smooth_phi_count(Lc), smooth_phi_count(Lp)
        n = int(lv[l + 1]["nbox"]) * nrhs
        e = {"child_L": Lc, "parent_L": Lp, "P_child": Pc, "P_parent": Pp, "items": n}
        for ant in (False, True):
            pi, po = (Pp, Pc) if ant else (Pc, Pp)
            r = G.FFTResampler(Lc, pi, po, anterpolate=ant)
            x = torch.randn(n, pi // 2, pi, dtype=torch.complex64, device="cuda")
            y = r(x)
            for _ in range(3):
                r(x, out=y)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                r(x, out=y)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            b = 8.0 * n * (pi // 2 * pi + po // 2 * po)
            key = "anterp" if ant else "interp"
            e[key + "_ms"] = round(ms, 4)
            e[key + "_GBs"] = round(b / (ms * 1e-3) / 1e9, 1)
            tot[ant] += ms
            byt[ant] += b
            del x, y, r
        out["pairs"].append(e)
    for ant, key in ((False, "interp"), (True, "anterp")):
        out[key + "_ms_total"] = round(tot[ant], 4)
        gbs = byt[ant] / max(tot[ant] * 1e-3, 1e-12) / 1e9
        out[key + "_hbm_frac"] = round(gbs / PEAK_HBM_GBS, 4)
    out["dense_m2m_ms_alone"] = dense_phases.get("m2m", {}).get("ms_alone")
    out["dense_l2l_ms_alone"] = dense_phases.get("l2l", {}).get("ms_alone")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="sphere262k")
    ap.add_argument("--nrhs", type=int, default=None)
    ap.add_argument("--bf16x3", action="store_true")
    ap.add_argument("--graph", action="store_true",
                    help="capture the matvec into a HIP graph and replay it")
    ap.add_argument("--one-stream", action="store_true",
                    help="every kernel on the caller's stream (no near/far overlap)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads (spheroid, 64 RHS, volume cloud)")
    ap.add_argument("--forms", default=None,
                    help="JSON object of kernel forms to take instead of autotuning, as "
                         "the bench line's \"forms\" prints them: per-level lists "
                         "(index = level - 1, -1 = none) for m2l, interp and anterp, and "
                         "p2p = [near-field fork point, M2L CU share in eighths, leaf "
                         "M2L late 0/1, near field in two halves 0/1]; used to "
                         "collect hardware counters of the forms a timed run chose")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one 256 MiB device-to-device copy first (a kernel of known "
                         "traffic for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the multi-GPU path is not part of this "
              "build (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2006_15367_amd import mlfma as G
    from paper_2006_15367_amd import workloads as W

    xyz, q = W.make(args.workload, nrhs=args.nrhs)
    R = 1 if q.ndim == 1 else q.shape[1]
    t0 = time.perf_counter()
    tree = G.Tree(xyz, W.LEAF_SIZE)
    t1 = time.perf_counter()
    ops = G.Operators(tree, W.K_WAVENUMBER, W.DIGITS, max_rhs=R, bf16x3=args.bf16x3,
                      graph=args.graph, one_stream=args.one_stream,
                      autotune=args.forms is None)
    if args.forms is not None:
        forms = json.loads(args.forms)
        for kern in ("m2l", "interp", "anterp"):
            for i, v in enumerate(forms.get(kern, [])):
                if v >= 0:
                    ops.set_variant(i + 1, v, kern)
        if "p2p" in forms and not args.one_stream and min(forms["p2p"]) >= 0:
            # [fork point, M2L CU share, leaf M2L late, near field halves]
            # as levels 0, 1, 2, 3
            for i, v in enumerate(forms["p2p"]):
                ops.set_variant(i, v, "p2p")
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    tinfo = tree.info()
    levels = ops.levels()
    qd = torch.from_numpy(np.ascontiguousarray(q.astype(np.complex64))).cuda()
    vd = torch.from_numpy(np.ascontiguousarray(np.conj(q).astype(np.complex64))).cuda()

    if args.copy_probe:
        src = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
        src.fill_(1.0)
        dst = src.clone()
        torch.cuda.synchronize()
        del src, dst
    # graph mode replays a captured graph, which needs a non-null stream
    st = torch.cuda.Stream() if args.graph else torch.cuda.current_stream()
    with torch.cuda.stream(st):
        for _ in range(args.warmup):
            phi = ops.matvec(qd, stream=st)
        torch.cuda.synchronize()
        # ten profiled (eager) steps, every kernel timed alone: per-phase
        # times and the dominant kernel
        # (128 launches a step: more than any workload's matvec makes, and
        # few enough events that creating them leaves the timed steps alone;
        # 4096 a step, 82k events created and destroyed right before the
        # timed region, slowed it by about 5 us a step)
        n_prof = 10
        ops.profile_begin(None, 128 * n_prof, serial=True)
        for _ in range(n_prof):
            ops.matvec(qd, stream=st)
        torch.cuda.synchronize()
        per_kernel = {k: (v[0] / n_prof, v[1] // n_prof) for k, v in ops.profile_end().items()}
        dominant = max(per_kernel, key=lambda k: per_kernel[k][0])
        launches = per_kernel[dominant][1]

        # timed region: K steps.  Eager mode times the dominant kernel's
        # launches with HIP events inside the timed region, in its last
        # tenth of the steps (a step whose launches record events runs about
        # 35 us longer on the 262k sphere, the side-stream schedule around
        # them disturbed; kept off the other nine tenths); graph mode times
        # them in an equal number of eager steps right after it.
        n_ev = max(1, args.steps // 10)
        # (a session of the same size before the timed region: the library
        # keeps its events, so the one started inside the loop creates none)
        n_rec = launches * (n_ev if not args.graph else args.steps) + 16
        ops.profile_begin([dominant], n_rec)
        ops.profile_end()
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for i in range(args.steps):
            if not args.graph and i == args.steps - n_ev:
                ops.profile_begin([dominant], n_rec)
            phi = ops.matvec(qd, stream=st)
        torch.cuda.synchronize()
        te = time.perf_counter()
        eager_ms = None
        if args.graph:
            ops.profile_begin([dominant], n_rec)
            te0 = time.perf_counter()
            for _ in range(args.steps):
                ops.matvec(qd, stream=st)
            torch.cuda.synchronize()
            eager_ms = (time.perf_counter() - te0) * 1e3 / args.steps
        dom = ops.profile_end()[dominant]
        ms_per_step = (te - ts) * 1e3 / args.steps
        # the same kernel timed alone: K more steps with every kernel on one
        # stream (in the timed steps it shares the device with concurrent work)
        ops.profile_begin([dominant], launches * args.steps + 16, serial=True)
        for _ in range(args.steps):
            ops.matvec(qd, stream=st)
        torch.cuda.synchronize()
        dom_alone = ops.profile_end()[dominant]

        # adjoint, timed the same way (no events)
        for _ in range(2):
            ops.adjoint(vd, stream=st)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(args.steps):
            psi = ops.adjoint(vd, stream=st)
        torch.cuda.synchronize()
        adj_ms = (time.perf_counter() - ta) * 1e3 / args.steps

        # iterative solve of (shift I + A) x = q by restarted GMRES on the
        # same operator (one right-hand side); the first call allocates the
        # Krylov workspace and is not timed
        gmres = None
        if R == 1:
            ops.solve(qd, GMRES_SHIFT, restart=30, max_iters=2, tol=1e-5, stream=st)
            torch.cuda.synchronize()
            tg = time.perf_counter()
            _, g_it, g_rr = ops.solve(qd, GMRES_SHIFT, restart=30, max_iters=300, tol=1e-5,
                                      stream=st)
            g_ms = (time.perf_counter() - tg) * 1e3
            gmres = {"system": "(shift I + A) x = q, shift = %gi" % GMRES_SHIFT.imag,
                     "restart": 30, "tol": 1e-5, "iterations": g_it,
                     "rel_residual": g_rr, "ms": round(g_ms, 3),
                     "ms_per_iteration": round(g_ms / max(1, g_it), 4),
                     "matvec_share": round(g_it * ms_per_step / g_ms, 3)}

    work = algorithmic_work(tinfo, levels, R, ops.variants("interp"), ops.variants("anterp"))
    ev_steps = args.steps if args.graph else n_ev  # steps whose launches the events timed
    rl = roofline(dominant, work[dominant], dom[0] / ev_steps, launches, args.bf16x3)
    alone = roofline(dominant, work[dominant], dom_alone[0] / args.steps, launches, args.bf16x3)
    rl["event_steps"] = ev_steps
    rl["alone"] = {k: alone[k] for k in ("achieved", "frac", "avg_launch_us", "ms_per_step")}
    rl["traffic"] = recorded_traffic(dominant, args.workload, R,
                                     ops.variants("m2l") if dominant == "m2l" else None)
    phases, floor_ms = phase_rooflines(work, {k: v[0] for k, v in per_kernel.items()},
                                       args.bf16x3)
    if rl["traffic"] is not None:
        rl["algorithmic_bytes_per_launch"] = round(work[dominant]["bytes"] / max(1, launches), 1)
    value = xyz.shape[0] * R / (ms_per_step * 1e-3)
    out = {
        "metric": "MLFMA matvec points/s at 1e-3 rel-L2 (+adjoint)",
        "value": round(value, 1), "unit": "points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 (fp32)" + (" + bf16x3 interpolation" if args.bf16x3 else ""),
        "data": "synthetic",
        "config": {"workload": args.workload, "n_points": int(xyz.shape[0]), "nrhs": R,
                   "k": W.K_WAVENUMBER, "leaf": W.LEAF_SIZE, "digits": W.DIGITS,
                   "levels": tinfo["n_levels"], "parallelism": "single GPU"},
        "adjoint": {"value": round(xyz.shape[0] * R / (adj_ms * 1e-3), 1),
                    "ms_per_step": round(adj_ms, 4)},
        "setup_s": {"tree": round(t1 - t0, 3), "operators": round(t2 - t1, 3)},
        "graph": bool(args.graph),
        "one_stream": bool(args.one_stream),
        "eager_ms_per_step": None if eager_ms is None else round(eager_ms, 4),
        "kernel_ms_one_step": {k: round(v[0], 4) for k, v in per_kernel.items()},
        "m2l_variant_per_level": ops.variants("m2l"),
        "near_field_fork": {0: "downward pass", 1: "start", 2: "after C2M",
                            3: "after the first M2M", 4: "after the second M2M"}.get(
            ops.variants("p2p")[0], "one stream"),
        "m2l_cu_share_eighths": ops.variants("p2p")[1],
        "leaf_m2l": {0: "beside the upward pass", 1: "during the downward pass"}.get(
            ops.variants("p2p")[2], "one stream"),
        "near_field_halves": ops.variants("p2p")[3],
        "onepass_interp_per_level": ops.variants("interp"),
        "onepass_anterp_per_level": ops.variants("anterp"),
        "forms": {k: ops.variants(k) for k in ("m2l", "interp", "anterp", "p2p")},
        "roofline": rl,
        "phases": phases,
        "whole_matvec": {"floor_ms": round(floor_ms, 5), "ms": round(ms_per_step, 4),
                         "frac": round(floor_ms / ms_per_step, 4),
                         "floor": "sum over phases of max(algorithmic bytes / 8 TB/s, "
                                  "algorithmic flops / compute peak)"},
        "gmres": gmres,
    }
    if not args.no_extras and args.workload in ("sphere262k", "sphere262k_r64") and \
            not args.graph and not args.bf16x3:
        try:
            out["fft_interpolation"] = fft_ablation(levels, R, phases)
        except Exception as ex:  # keep the headline line whatever happens here
            out["fft_interpolation"] = {"error": "%s: %s" % (type(ex).__name__, ex)}
    if not args.no_extras and args.workload == "sphere262k" and not args.graph:
        out["extra_workloads"] = extra_workloads(ms_per_step, ops.memory()["operator_bytes"])
    if not args.no_cpu_baseline:
        phi_np = phi.cpu().numpy().astype(np.complex128)
        out["cpu_baseline"] = cpu_baseline(xyz, q.astype(np.complex128), phi_np)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
