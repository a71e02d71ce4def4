#!/usr/bin/env python3
"""Benchmark of the sweep of the lower-bound iteration for gamma_{2,2}.

Workload: sigma = d = 2, l = 16 (2^32 table indices, of which the 2^31 with
string-1 head 0 are stored: the complement symmetry of Sec. 3.3), FP32 sweeps
renormalised by entry 0, with an FP64 round-down certificate every 64 sweeps
(the largest-r certificate of the newest table: one pass, no R pass).
One step is one certificate period: 64 sweeps + one certificate.  The
reported value is table updates per second (2^32 updates per sweep, one per
index) over the K timed steps, with the ring already resident in HBM.

The zero-start ring is symmetric in the two strings, so the sweep runs the
exchange-folded kernel (one tuple of each exchanged pair computed and
stored; the table is completed only where it is read as a whole), and it
reads the branch means of the lags (lcsb_bind_means: one advance-a,
advance-b or all-advance mean per branch instead of its 2 or 4 entries),
writing the entries of the new table on the last two sweeps of each period.

Also printed in the same JSON line:
  roofline      the sweep kernel's algorithmic bytes per launch (6 B per
                stored FP32 entry: lag 1 and lag 2 read, and the new table
                written, at one entry of each exchanged pair; 3 B per
                update) over its average launch time (the branch-mean sweep
                moves fewer bytes than this: see traffic)
                (traffic_GBps / traffic_frac: the same with the measured HBM
                bytes), from HIP events on the stream
                the library launches on, against the 8 TB/s HBM peak; traffic
                is the rocprofv3-measured HBM bytes per launch when a counter
                summary for the current kernel source is committed, else null
  cpu_baseline  the CPU oracle on this host, one sweep over a bounded sample
                of the same table
  time_to_bound wall time to a certified bound within 1e-9 of the converged
                plain FP64 bound, for plain FP64, for FP32 + FP64 polish, and
                for the same started from the learned warm start
"""
import argparse
import gc
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "updates/s at σ=2,d=2,h=16; time to certified bound, plain vs mixed+learned"
PMC_SUMMARY = os.path.join(ROOT, "profiles", "sweep_s2d2_f32_h16_pmc.json")
PMC_SUMMARY_F64_H14 = os.path.join(ROOT, "profiles", "sweep_s2d2_f64_h14_pmc.json")
SWEEP_SRC = os.path.join(ROOT, "paper_2407_10925_amd", "csrc", "sweep.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--h", type=int, default=16)
    p.add_argument("--sigma", type=int, default=2, help="alphabet size (counter-collection modes)")
    p.add_argument("--d", type=int, default=2, help="number of strings (counter-collection modes)")
    p.add_argument("--dtype", default="f32", choices=["f32", "f64"],
                   help="table type (counter-collection modes)")
    p.add_argument("--cadence", type=int, default=64)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--cpu-sample-log2", type=int, default=24)
    p.add_argument("--no-ttb", action="store_true", help="skip the time-to-bound runs")
    p.add_argument("--train-steps", type=int, default=1000)
    p.add_argument("--no-means", action="store_true",
                   help="with --profile-sweeps: the entry-reading sweep (no branch-mean buffers)")
    p.add_argument("--profile-sweeps", type=int, default=0,
                   help="only run this many FP32 sweeps from zero (for counter collection)")
    p.add_argument("--configs", action="store_true",
                   help="only time one sweep and one certificate for every configuration")
    p.add_argument("--copy-gib", type=float, default=0.0,
                   help="only run one plain device copy of this many GiB (counter calibration)")
    p.add_argument("--profile-seed", action="store_true",
                   help="only seed an FP32 ring from an (untrained) warm-start network, twice")
    p.add_argument("--profile-train", type=int, default=0,
                   help="only generate the warm-start training tables and run this many steps")
    p.add_argument("--train-batch", type=int, default=8192, help="batch of --profile-train")
    p.add_argument("--converge", type=int, default=0, metavar="L",
                   help="only run plain FP64 at (--sigma, --d, l = L) to convergence, then FP32 + "
                        "FP64 polish to the same bound in the same memory")
    p.add_argument("--two-array-f32", type=int, default=0, metavar="L",
                   help="only the FP32 two-array iteration from zero at sigma=d=2, l=L, "
                        "certified every 16 sweeps (the largest-r certificate) for --max-sweeps")
    p.add_argument("--max-sweeps", type=int, default=480)
    p.add_argument("--iteration", default="ring", choices=["ring", "two_array"],
                   help="iteration of --converge")
    p.add_argument("--certificate", default="feasible", choices=["feasible", "optimal"],
                   help="certificate of --converge")
    p.add_argument("--packed", type=int, default=0, metavar="L",
                   help="only sigma=d=2 at l=L on exchange-packed tables: plain FP64 two-array "
                        "to convergence, then FP32 + FP64 polish in the same memory")
    p.add_argument("--seed-ceiling", action="store_true",
                   help="only measure what a warm start of known error saves at sigma=d=2, "
                        "l=--h (the converged table plus noise, and the trained network)")
    p.add_argument("--profile-certify", action="store_true",
                   help="only run 8 sweeps from zero and two certificates (counter collection)")
    return p.parse_args()


def sweep_source_hash():
    with open(SWEEP_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(path=PMC_SUMMARY):
    """HBM bytes per sweep launch from a committed rocprofv3 counter summary,
    or None when absent or taken on a different kernel source."""
    try:
        with open(path) as f:
            s = json.load(f)
    except (OSError, ValueError):
        return None
    if s.get("sweep_hip_sha256") != sweep_source_hash():
        return None
    return s.get("hbm_bytes_per_launch")


def host_description():
    """CPU model, logical CPUs, the CPUs this process may run on, and RAM."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    mem = None
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    mem = round(int(line.split()[1]) / 2**20, 1)
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)), "ram_GiB": mem}


def cpu_baseline(pk, h, log2_sample, max_threads=16):
    """The oracle on this host's cores: one sweep over every 2^(2h - s)-th
    entry of an l = h FP32 ring filled with seeded values, first on one
    thread, then split into contiguous index ranges over `threads` threads
    (the oracle itself stays single-threaded per call; ctypes releases the
    interpreter lock, so the calls run in parallel and give the same bits).
    Also the whole C1 run (sigma = d = 2, l = 6, FP64, 200 sweeps from zero,
    a certificate after every sweep) on the oracle and on the GPU."""
    import numpy as np
    import torch
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import seeded_inputs as si

    n = 4 ** h
    log(f"cpu baseline: generating a seeded l={h} FP32 ring")
    lags = []
    for k in range(2):
        t = si.table(2, 2, h, seed=100 + k, dtype=torch.float32, device="cuda")
        lags.append(t.cpu().numpy())
        del t
    torch.cuda.empty_cache()
    count = min(n, 1 << log2_sample)
    idx = np.arange(0, n, n // count, dtype=np.uint64)[:count]
    oracle.lib()
    log(f"cpu baseline: oracle sweep over {count} sampled entries, one thread")
    t0 = time.perf_counter()
    ref = oracle.sweep_at_tables(2, 2, h, lags, idx)
    dt1 = time.perf_counter() - t0
    threads = max(1, min(max_threads, len(os.sched_getaffinity(0))))
    parts = np.array_split(idx, threads)
    log(f"cpu baseline: the same over {threads} threads")
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        outs = list(ex.map(lambda part: oracle.sweep_at_tables(2, 2, h, lags, part), parts))
    dtn = time.perf_counter() - t0
    if not np.array_equal(np.concatenate(outs), ref):
        raise RuntimeError("threaded oracle sweep differs from the single-threaded one")
    del lags
    # C1: the whole small run, oracle and GPU
    t0 = time.perf_counter()
    best_o, _, _ = oracle.feasible_triplet(2, 2, 6, 200, 1)
    c1_oracle = time.perf_counter() - t0
    L = pk.Lcsb(2, 2, 6, "f64")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L.init_zero()
    _, best_g, _, _ = L.run(1, max_sweeps=200)
    torch.cuda.synchronize()
    c1_gpu = time.perf_counter() - t0
    if best_g["bound"] != best_o["bound"]:
        raise RuntimeError("C1: GPU and oracle best bounds differ")
    # one sweep of the plain at-scale configuration (sigma = d = 2, l = 14:
    # 2^28 updates), extrapolated from the two rates measured above
    c2 = {"updates_per_sweep": 4 ** 14,
          "one_thread_s": round(4 ** 14 * dt1 / count, 1),
          "all_threads_s": round(4 ** 14 * dtn / count, 1),
          "note": "scaled from the sampled l = 16 sweep rates, an upper estimate (the "
                  "oracle decodes each tuple in O(l) steps); not run whole"}
    return {"value": count / dtn, "unit": "updates/s", "cores": threads, "kind": "oracle",
            "sample": f"one sweep at {count} entries (every {n // count}th index) of the "
                      f"sigma=d=2, l={h} table, FP32 ring read as FP64, {threads} threads over "
                      f"contiguous index ranges ({dtn:.2f} s); one thread: {dt1:.1f} s",
            "single_thread_value": count / dt1,
            "host": host_description(),
            "c2_sigma2_d2_l14_one_sweep": c2,
            "c1_sigma2_d2_l6_200_sweeps_certified_each": {
                "oracle_s": round(c1_oracle, 4), "gpu_s": round(c1_gpu, 4),
                "best_bound": best_o["bound"]}}


# Certification policy shared by every time-to-bound run (none uses B):
TTB_CADENCE = 16      # plain FP64 and FP32 phases: sweeps between certificates
SWITCH_GAIN = 2e-5    # leave FP32 once a positive best bound gains less than this in a period
POLISH_FIRST = 32     # FP64 sweeps after the upcast before the first polish certificate
POLISH_CADENCE = 8    # then a certificate every this many FP64 sweeps
MAX_SWEEPS = 1600


def fp32_until_floor(S, certificate="feasible"):
    """FP32 sweeps with a certificate every TTB_CADENCE sweeps until the best
    bound is positive and gains less than SWITCH_GAIN over one period (the
    FP32 error floor), as one lcsb_run.  Returns (cur, best, certificates)."""
    cur, best, certs, _ = S.run(TTB_CADENCE, max_sweeps=MAX_SWEEPS, min_gain=SWITCH_GAIN,
                                certificate=certificate)
    return cur, best, certs


def polish(P, S, best, target, certificate="feasible"):
    """Upcast the FP32 ring into P and continue in FP64 (first certificate
    after POLISH_FIRST sweeps, then every POLISH_CADENCE) until the best
    certified bound reaches target.  Returns (FP64 sweeps, certificates, best)."""
    if best["bound"] >= target:
        return 0, 0, best
    P.upcast(S)  # the best certificate of the FP32 run moves over
    start = P.status()[0]
    _, best, certs, _ = P.run(POLISH_CADENCE, first=POLISH_FIRST, max_sweeps=MAX_SWEEPS,
                              target=target, certificate=certificate)
    return P.status()[0] - start, certs, best


def uses_means(iteration, sigma, d):
    """Branch-mean buffers serve the rings and two-array pairs of sigma = 2
    (d = 2, 3) and sigma = 4 (d = 2)."""
    if iteration not in ("ring", "two_array"):
        return False
    return (sigma == 2 and d in (2, 3)) or (sigma == 4 and d == 2)


def new_ring(pk, sigma, d, h, dtype, iteration="ring", means=True, **kw):
    """An Lcsb with branch-mean buffers where its shape takes them and they fit
    beside its tables (`L.means` is then non-empty), else without them."""
    import torch
    if means and uses_means(iteration, sigma, d):
        L = None
        try:
            L = pk.Lcsb(sigma, d, h, dtype, iteration=iteration, means=True, **kw)
        except torch.cuda.OutOfMemoryError:
            pass
        if L is not None:
            return L
        gc.collect()  # the partial context, outside the handler
        torch.cuda.empty_cache()
    return pk.Lcsb(sigma, d, h, dtype, iteration=iteration, **kw)


def plain_run(pk, h, target, iteration="ring", certificate="feasible", sigma=2, d=2):
    """FP64 from zero, a certificate every TTB_CADENCE sweeps, until the best
    bound reaches target (one lcsb_run, timed from the init call)."""
    import torch
    P = new_ring(pk, sigma, d, h, "f64", iteration)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.init_zero()
    cur, best, certs, _ = P.run(TTB_CADENCE, max_sweeps=MAX_SWEEPS, target=target,
                                certificate=certificate)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {"seconds": round(dt, 4), "sweeps": cur["sweep"], "certificates": certs,
           "bound": best["bound"], "reached": best["bound"] >= target,
           "iteration": iteration, "certificate": certificate}
    del P
    torch.cuda.empty_cache()
    return out


def mixed_run(pk, h, target, iteration="ring", certificate="feasible", sigma=2, d=2):
    """FP32 from zero to its error floor, then the FP64 polish to target, the
    FP32 tables inside the FP64 buffers (widened in place)."""
    import torch
    P = new_ring(pk, sigma, d, h, "f64", iteration)
    M = new_ring(pk, sigma, d, h, "f32", iteration, bufs=[b.view(torch.float32) for b in P.bufs])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    M.init_zero()
    cur, best, certs32 = fp32_until_floor(M, certificate)
    sweeps32 = cur["sweep"]
    sweeps64, certs64, best = polish(P, M, best, target, certificate)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {"seconds": round(dt, 4), "sweeps_f32": sweeps32, "sweeps_f64": sweeps64,
           "certificates": certs32 + certs64, "bound": best["bound"],
           "reached": best["bound"] >= target, "iteration": iteration,
           "certificate": certificate}
    del P, M
    torch.cuda.empty_cache()
    return out


def algorithmic_bytes(L, elem):
    """Bytes one sigma = d = 2 sweep must move: lag 1 and lag 2 read once and
    the new stored table written once; on an exchange-symmetric ring one
    entry of each exchanged pair carries the information, so each lag is
    read, and the new table written, at half its stored entries."""
    if L.swap_symmetric():
        return 3 * elem * L.stored // 2
    return 3 * elem * L.stored


def sweep_kernel(L, ctype):
    """Name of the sigma = d = 2 sweep kernel a ring runs."""
    if L.swap_symmetric() and L.means:
        return f"sweep_s2d2_means<{ctype}, false>"
    return f"sweep_s2d2<{ctype}, {'true' if L.swap_symmetric() else 'false'}, false>"


def fp64_sweep(pk, h, sweeps=32):
    """The plain FP64 sweep (bit-identical to the oracle) at sigma = d = 2,
    l = h from zero: average launch time from HIP events on the library's
    stream, against the HBM peak (12 algorithmic bytes per stored entry)."""
    import torch
    L = pk.Lcsb(2, 2, h, "f64", means=True)
    L.init_zero()
    L.iterate(8)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    L.iterate(sweeps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / sweeps
    n = 4 ** h
    algo = algorithmic_bytes(L, 8)
    kernel = sweep_kernel(L, "double")
    gbs = algo / ms / 1e6
    del L
    torch.cuda.empty_cache()
    out = {"workload": f"sigma=2 d=2 l={h}: {n} FP64 table indices ({n // 2} stored)",
           "bound": "hbm",
           "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(gbs / HBM_PEAK_GBS, 4), "avg_launch_ms": round(ms, 4),
           "kernel": kernel, "sweeps_per_launch_group": sweeps,
           "algorithmic_bytes_per_launch": algo,
           "updates_per_s": n / ms * 1e3, "traffic": None}
    traffic = measured_traffic(PMC_SUMMARY_F64_H14) if h == 14 else None
    if traffic is not None:  # rocprofv3-measured HBM bytes per launch, at this launch time
        out["traffic"] = traffic
        out["traffic_GBps"] = round(traffic / ms / 1e6, 1)
        out["traffic_frac"] = round(traffic / ms / 1e6 / HBM_PEAK_GBS, 4)
    return out


def fp32_error(P, S, chunk=1 << 28):
    """Largest per-entry difference between the FP32 table of S and the FP64
    table of P, both taken relative to their entry 0, over the FP64 table's
    spread (max - min); computed in chunks on the device."""
    import torch
    t64, _ = P.lag(1)
    t32, _ = S.lag(1)  # the FP32 offset cancels in the difference to entry 0
    r64, r32 = float(t64[0]), float(t32[0])
    err, lo, hi = 0.0, math.inf, -math.inf
    for a in range(0, t64.numel(), chunk):
        x = t64[a:a + chunk] - r64
        y = t32[a:a + chunk].double() - r32
        err = max(err, float((x - y).abs().max()))
        lo, hi = min(lo, float(x.min())), max(hi, float(x.max()))
        del x, y
    return err / (hi - lo), hi - lo


def time_to_bound(pk, h, train_steps=1000):
    """Wall time from the init call to the first certificate within 1e-9 of
    the converged plain FP64 bound B (certificates, upcast and seeding
    included).  Every run is driven by lcsb_run.

    B:       FP64 from zero, a certificate every TTB_CADENCE sweeps, until
             consecutive certificates move by less than 1e-10 (untimed).
    plain:   FP64 from zero, a certificate every TTB_CADENCE sweeps, until the
             best bound reaches B - 1e-9.
    mixed:   FP32 from zero until its error floor (fp32_until_floor), then the
             FP64 polish (polish) until the best bound reaches B - 1e-9.
    learned: as mixed, from the warm-start network's seed (learned_run).

    Each run also reports the algorithmic bytes of its sweeps over its whole
    wall time against the HBM peak (certificates, upcast and seeding count
    as time, not as bytes: a lower bound on the HBM use of the run).
    """
    import torch
    out = {}
    P = pk.Lcsb(2, 2, h, "f64", means=True)
    P.init_zero()
    alg64 = algorithmic_bytes(P, 8)      # every ring here is exchange-symmetric
    alg32 = alg64 // 2

    def hbm(sweeps32, sweeps64, seconds):
        tbps = (sweeps32 * alg32 + sweeps64 * alg64) / seconds / 1e12
        return {"sweep_algorithmic_TBps": round(tbps, 3),
                "roofline_frac": round(tbps * 1e3 / HBM_PEAK_GBS, 4)}

    cur, best, _, why = P.run(TTB_CADENCE, max_sweeps=MAX_SWEEPS, stop_delta=1e-10)
    B = best["bound"]
    target = B - 1e-9
    converged_after = cur["sweep"]
    log(f"converged plain FP64 bound B = {B:.12f} after {converged_after} sweeps ({why})")

    M = pk.Lcsb(2, 2, h, "f32", means=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    M.init_zero()
    cur, best, certs32 = fp32_until_floor(M)
    sweeps32 = cur["sweep"]
    t_switch = time.perf_counter() - t0
    # outside the timed span: the FP32 table at its floor against the FP64
    # table after as many sweeps from the same zero start (the polish below
    # overwrites P's ring)
    P.init_zero()
    P.iterate(sweeps32)
    rel_err, spread = fp32_error(P, M)
    log(f"FP32 table at its floor vs FP64 after the same {sweeps32} sweeps: max |difference| / "
        f"spread = {rel_err:.3e} (spread {spread:.4f})")
    t0 += time.perf_counter() - t0 - t_switch
    sweeps64, certs64, best = polish(P, M, best, target)
    torch.cuda.synchronize()
    t_mixed = time.perf_counter() - t0
    out["mixed_f32_polish"] = {"seconds": round(t_mixed, 4), "sweeps_f32": sweeps32,
                               "sweeps_f64": sweeps64, "certificates": certs32 + certs64,
                               "switch_after_s": round(t_switch, 4), "bound": best["bound"],
                               "reached": best["bound"] >= target,
                               "fp32_table_max_error_over_spread": rel_err,
                               "fp32_error_reference": f"FP64 ring after the same {sweeps32} sweeps from zero",
                               "fp64_table_spread": spread, **hbm(sweeps32, sweeps64, t_mixed)}
    log(f"time to bound, FP32 + FP64 polish: {t_mixed:.3f} s, {sweeps32} FP32 + "
        f"{sweeps64} FP64 sweeps, bound {best['bound']:.12f}")
    del M
    torch.cuda.empty_cache()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.init_zero()
    cur, best, certs, _ = P.run(TTB_CADENCE, max_sweeps=MAX_SWEEPS, target=target)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    out["plain_f64"] = {"seconds": round(t_plain, 4), "sweeps": cur["sweep"], "certificates": certs,
                        "bound": B, "converged_after_sweeps": converged_after,
                        "certificate_every": TTB_CADENCE, **hbm(0, cur["sweep"], t_plain)}
    log(f"time to bound, plain FP64: {t_plain:.3f} s, {cur['sweep']} sweeps, bound {B:.12f}")

    out["mixed_learned"] = learned_run(pk, h, P, target, train_steps)
    ml = out["mixed_learned"]
    ml.update(hbm(ml["sweeps_f32"], ml["sweeps_f64"], ml["seconds"]))
    del P
    torch.cuda.empty_cache()
    # the same runs with the largest-r certificate, on the ring and on the
    # two-array iteration
    for name, fn, it in (("plain_f64_optimal", plain_run, "ring"),
                         ("mixed_f32_polish_optimal", mixed_run, "ring"),
                         ("two_array_f64_optimal", plain_run, "two_array"),
                         ("two_array_mixed_optimal", mixed_run, "two_array")):
        r = fn(pk, h, target, iteration=it, certificate="optimal")
        r.update(hbm(r.get("sweeps_f32", 0), r.get("sweeps_f64", r.get("sweeps", 0)),
                     r["seconds"]))
        out[name] = r
        log(f"time to bound, {name}: {r['seconds']:.3f} s, bound {r['bound']:.12f}")
    out["policy"] = {"certificate_every": TTB_CADENCE, "switch_gain": SWITCH_GAIN,
                     "polish_first": POLISH_FIRST, "polish_every": POLISH_CADENCE,
                     "driver": "lcsb_run"}
    runs = {k: v for k, v in out.items() if isinstance(v, dict) and "seconds" in v}
    fastest = min(runs, key=lambda k: runs[k]["seconds"])
    out["fastest"] = {"run": fastest, "seconds": runs[fastest]["seconds"],
                      "vs_plain_f64": round(runs["plain_f64"]["seconds"] / runs[fastest]["seconds"], 3)}
    return out


def train_network(pk, h, train_steps):
    """The warm-start network for l = h.  Training data: FP32 tables at
    l = h-4, h-3, h-2 run from zero to their error floor (fp32_until_floor);
    training: `train_steps` Adam steps on batches of 8192 drawn from those
    tables in turn, cosine learning-rate decay.  Returns (network, rate R of
    the l = h-2 run, data seconds, training seconds, last batch loss)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tables = []
    for hh in (h - 4, h - 3, h - 2):
        T = pk.Lcsb(2, 2, hh, "f32")
        T.init_zero()
        cur, _, _ = fp32_until_floor(T)
        tables.append((hh, T, T.lag(1)[0]))  # lag() reads the offset back: once, not per step
    rate = cur["R"]
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    M = pk.Mlp(batch=8192, seed=2407)
    t1 = time.perf_counter()
    lr0 = 2e-3
    for step in range(train_steps):
        hh, _, table = tables[step % 3]
        lr = lr0 * 0.5 * (1 + math.cos(math.pi * step / train_steps))
        M.train_step(table, hh, seed=10925 + step, lr=lr)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    loss = M.loss_dev.item()
    del tables
    torch.cuda.empty_cache()
    log(f"warm start: data {t_data:.2f} s, training {t_train:.2f} s ({train_steps} steps), "
        f"last batch loss {loss:.3e}")
    return M, rate, t_data, t_train, loss


def learned_run(pk, h, P, target, train_steps):
    """FP32 + FP64 polish started from the warm-start network (train_network),
    seeded with the rate of its l = h-2 training run.  Times are reported
    without and with data generation and training."""
    import torch
    M, rate, t_data, t_train, loss = train_network(pk, h, train_steps)
    S = pk.Lcsb(2, 2, h, "f32", means=True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    S.init_seed_mlp(M, rate)
    torch.cuda.synchronize()
    t_seed = time.perf_counter() - t2
    cur, best, certs32 = fp32_until_floor(S)
    sweeps32 = cur["sweep"]
    sweeps64, certs64, best = polish(P, S, best, target)
    torch.cuda.synchronize()
    t_run = time.perf_counter() - t2
    res = {"seconds": round(t_run, 4), "seconds_with_training": round(t_run + t_data + t_train, 4),
           "data_s": round(t_data, 4), "training_s": round(t_train, 4), "train_steps": train_steps,
           "last_batch_loss": loss, "seed_s": round(t_seed, 4),
           "seed_tflops": round(MLP_FLOP * seed_evaluations(h) / t_seed / 1e12, 1),
           "sweeps_f32": sweeps32, "sweeps_f64": sweeps64, "certificates": certs32 + certs64,
           "bound": best["bound"], "reached": best["bound"] >= target}
    log(f"time to bound, learned + FP32 + FP64 polish: {t_run:.3f} s ({t_seed:.3f} s seed), "
        f"{sweeps32} FP32 + {sweeps64} FP64 sweeps, bound {best['bound']:.12f}")
    del S, M
    torch.cuda.empty_cache()
    return res


def _exchange_noise(h, lo, hi, device):
    """Uniform noise in [-1, 1) for the stored sigma = d = 2 indices lo..hi-1,
    equal on the two members of every pair under the exchange of the strings
    (a function of the lower representative), from a SplitMix64 hash of it."""
    import torch
    i = torch.arange(lo, hi, dtype=torch.int64, device=device)
    odd = (1 << (2 * h)) // 3 * 2        # string-1 bits (0b1010...)
    even = odd >> 1                      # string-2 bits (0b0101...)
    e = ((i & odd) >> 1) | ((i & even) << 1)
    top = 1 << (2 * h - 1)
    e = torch.where(e & top != 0, e ^ ((1 << (2 * h)) - 1), e)  # its complement-folded image
    c = torch.minimum(i, e)
    m64 = (1 << 64) - 1

    def s64(x):
        x &= m64
        return x - (1 << 64) if x >= 1 << 63 else x

    def lsr(z, k):
        return (z >> k) & ((1 << (64 - k)) - 1)
    z = (c + 1) * s64(0x9E3779B97F4A7C15)
    z = (z ^ lsr(z, 30)) * s64(0xBF58476D1CE4E5B9)
    z = (z ^ lsr(z, 27)) * s64(0x94D049BB133111EB)
    z = z ^ lsr(z, 31)
    return lsr(z, 11).to(torch.float64) * 2.0 ** -52 - 1.0


def seed_ceiling(pk, h, train_steps, rms_list=(0.0, 1e-4, 1e-3, 3e-3, 1e-2, 3e-2)):
    """What a warm start can save at sigma = d = 2, l = h.  The seed is the
    converged FP64 table (relative to entry 0) plus exchange-symmetric noise
    of a given RMS, loaded as an FP32 ring with the converged R; for each RMS,
    for the zero start and for the trained network's seed: FP32 sweeps to a
    largest-r certificate within 1e-5 of the converged bound B (certified
    every 4 sweeps), and the wall time of the standard mixed policy
    (fp32_until_floor, then polish) to B - 1e-9 from the loaded ring (loading
    and seeding not included)."""
    import torch
    P = pk.Lcsb(2, 2, h, "f64")
    P.init_zero()
    cur, best, _, _ = P.run(TTB_CADENCE, max_sweeps=MAX_SWEEPS, stop_delta=1e-10)
    B, R = best["bound"], cur["R"]
    u, _ = P.lag(1)
    x = (u - u[0]).float()             # the converged table relative to entry 0
    spread = float(x.max() - x.min())
    log(f"converged B = {B:.12f}, R = {R:.12f}, spread {spread:.4f}")
    S = pk.Lcsb(2, 2, h, "f32")
    chunk = 1 << 27
    rows = []

    def measure(label, load, rms):
        load()
        cur, _, _, _ = S.run(4, max_sweeps=MAX_SWEEPS, target=B - 1e-5, certificate="optimal")
        near = cur["sweep"]
        load()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cur, best, c32 = fp32_until_floor(S)
        s64, c64, best = polish(P, S, best, B - 1e-9)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rows.append({"start": label, "seed_rms": rms, "sweeps_f32_to_1e-5": near,
                     "mixed_seconds": round(dt, 4), "sweeps_f32": cur["sweep"],
                     "sweeps_f64": s64, "reached": best["bound"] >= B - 1e-9})
        log(f"{label}: rms {rms}: {near} FP32 sweeps to B - 1e-5; mixed {dt:.3f} s "
            f"({cur['sweep']} FP32 + {s64} FP64 sweeps)")

    measure("zero", S.init_zero, None)
    seed = torch.empty_like(x)
    for rms in rms_list:
        for lo in range(0, x.numel(), chunk):
            hi = min(x.numel(), lo + chunk)
            seed[lo:hi] = x[lo:hi] + (rms * math.sqrt(3.0)
                                      * _exchange_noise(h, lo, hi, x.device)).float()
        measure("converged + noise", lambda: S.load_ring([seed, seed], [0.0, -R]), rms)
    del seed
    torch.cuda.empty_cache()
    M, rate, _, _, loss = train_network(pk, h, train_steps)
    S.init_seed_mlp(M, rate)
    t, off = S.lag(1)
    sq, mean_d = 0.0, 0.0
    ref = float(t[0]) + off
    for lo in range(0, x.numel(), chunk):
        dlt = (t[lo:lo + chunk].double() + (off - ref)) - x[lo:lo + chunk].double()
        mean_d += float(dlt.sum())
        sq += float((dlt * dlt).sum())
    mean_d /= x.numel()
    net_rms = math.sqrt(max(sq / x.numel() - mean_d * mean_d, 0.0))
    log(f"network seed: RMS error {net_rms:.3e} against the converged table (loss {loss:.3e})")
    measure("network", lambda: S.init_seed_mlp(M, rate), round(net_rms, 6))
    print(json.dumps({"seed_ceiling": {"h": h, "B": B, "R": R, "table_spread": spread,
                                       "runs": rows}}), flush=True)


CONFIGS = [  # (sigma, d, l, dtype)
    (2, 2, 6, "f64"), (2, 2, 14, "f64"), (2, 2, 16, "f32"), (2, 2, 16, "f64"),
    (4, 2, 8, "f32"), (2, 3, 10, "f32"), (4, 2, 8, "f64"), (2, 3, 10, "f64"),
    (2, 2, 17, "f32"), (2, 2, 17, "f64"),
]


GENERALITY = [(4, 2, 8, "f32"), (2, 3, 10, "f32"), (4, 2, 8, "f64"), (2, 3, 10, "f64")]


def designed_bytes(sigma, d, n, elem, means, folded, reps=64):
    """HBM bytes per sweep that the kernel a configuration runs is designed to
    move (values x elem).  Branch-mean sweeps: sigma = d = 2 reads Ma (n/4)
    and Mab at the lower prefixes (n/16) and writes both; d = 3 reads 13/32 n
    and writes 19/32 n; sigma = 4 reads M4a (n/16) and M4ab (n/128) and writes
    both; each also writes its stored entries at one per exchanged pair on the
    last d sweeps of a `reps`-sweep call.  Entry sweeps: the algorithmic bytes
    times their designed re-read (lag 1 twice: 4/3 for d = 2; 1.625 for d = 3)."""
    stored = n // (2 if sigma == 2 else 4)
    lower = stored // 2 if folded else stored
    if means:
        vals = {(2, 2): 2 * 5 * n / 16, (2, 3): n, (4, 2): 2 * 9 * n / 128}[(sigma, d)]
        return (vals + d / reps * lower) * elem
    return (d + 1) * lower * elem * (1.625 if d == 3 else 4 / 3)


def config_table(pk, configs=None, emit=True):
    """Average sweep and certificate time per configuration (HIP events; 64
    sweeps in one call, as a certificate period of the benchmark), with the
    sweep's algorithmic bytes against the HBM peak.  Rings of the shapes
    with branch-mean tables sweep from them where they fit beside the ring."""
    import torch
    rows = []
    for sigma, d, h, dt in (CONFIGS if configs is None else configs):
        L = new_ring(pk, sigma, d, h, dt)  # without means where they do not fit
        means = bool(L.means)
        L.init_zero()
        L.iterate(8)
        stream = torch.cuda.current_stream()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        reps = 64
        e[0].record(stream)
        L.iterate(reps)
        e[1].record(stream)
        e[2].record(stream)
        L.certify()
        e[3].record(stream)
        e[4].record(stream)
        L.certify_optimal()
        e[5].record(stream)
        torch.cuda.synchronize()
        sweep_ms = e[0].elapsed_time(e[1]) / reps
        cert_ms = e[2].elapsed_time(e[3])
        opt_ms = e[4].elapsed_time(e[5])
        elem = 8 if dt == "f64" else 4
        folded = L.swap_symmetric()  # exchange-folded: every table at one entry per pair
        algo = (d + 1) * elem * L.stored // (2 if folded else 1)
        kern = designed_bytes(sigma, d, L.n, elem, means, folded, reps)
        # algorithmic: each lag read once and one table written (what an
        # entry-reading sweep moves at least; a branch-mean sweep moves less,
        # so its fraction can pass 1); designed: what the kernel that ran moves
        rows.append({"sigma": sigma, "d": d, "l": h, "dtype": dt, "entries": L.n,
                     "exchange_folded": folded, "branch_means": means,
                     "sweep_ms": round(sweep_ms, 4), "certificate_ms": round(cert_ms, 3),
                     "optimal_certificate_ms": round(opt_ms, 3),
                     "algorithmic_GBps": round(algo / sweep_ms / 1e6, 1),
                     "frac_of_peak": round(algo / sweep_ms / 1e6 / HBM_PEAK_GBS, 4),
                     "designed_GB": round(kern / 1e9, 4),
                     "designed_GBps": round(kern / sweep_ms / 1e6, 1),
                     "designed_frac_of_peak": round(kern / sweep_ms / 1e6 / HBM_PEAK_GBS, 4),
                     "updates_per_s": L.n / sweep_ms * 1e3})
        log(json.dumps(rows[-1]))
        del L
        torch.cuda.empty_cache()
    if emit:
        print(json.dumps({"configs": rows}), flush=True)
    return rows


def profile_only(pk, h, sweeps, sigma=2, d=2, dtype="f32", means=True):
    """Only `sweeps` sweeps from zero at (sigma, d, l = h), for counters, as one
    lcsb_iterate call (the sigma = d = 2 ring with its branch-mean buffers
    unless means is False)."""
    import torch
    L = new_ring(pk, sigma, d, h, dtype, means=means)
    L.init_zero()
    L.iterate(sweeps)
    torch.cuda.synchronize()
    log(f"ran {sweeps} {dtype} sweeps at sigma={sigma} d={d} l={h}")


MLP_FLOP = 2 * (32 * 256 + 2 * 256 * 256 + 256)  # multiply-adds of one network evaluation, x2


def seed_evaluations(h):
    """Network evaluations of one seeding: one per orbit of exchanging the
    strings and complementing both, (4^l + 2^(l+1)) / 4."""
    return ((1 << h) + 2) << (h - 2)


def seed_only(pk, h):
    """Two seedings of an l = h FP32 ring by the warm-start network (random
    initial weights: the same work as a trained one), the second one timed."""
    import torch
    M = pk.Mlp(batch=256, seed=1)
    S = pk.Lcsb(2, 2, h, "f32")
    S.init_seed_mlp(M, 0.39)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.init_seed_mlp(M, 0.39)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    flop = MLP_FLOP * seed_evaluations(h)
    log(f"seed at l={h}: {dt * 1e3:.1f} ms, {flop / dt / 1e12:.0f} TFLOP/s over "
        f"{seed_evaluations(h)} orbit representatives")


def train_only(pk, h, steps, batch=8192):
    """Training tables at l = h-4..h-2 (FP32 to their floor), then `steps`
    training steps of the warm-start network, timed."""
    import torch
    tables = []
    for hh in (h - 4, h - 3, h - 2):
        T = pk.Lcsb(2, 2, hh, "f32")
        T.init_zero()
        fp32_until_floor(T)
        tables.append((hh, T, T.lag(1)[0]))
    M = pk.Mlp(batch=batch, seed=2407)
    M.train_step(tables[0][2], tables[0][0], seed=1, lr=1e-3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for step in range(steps):
        hh, _, table = tables[step % 3]
        M.train_step(table, hh, seed=10925 + step, lr=1e-3)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    flop = 3 * MLP_FLOP * batch * steps  # forward + backward (twice the forward)
    log(f"training: {steps} steps of batch {batch} in {dt:.3f} s, {dt / steps * 1e3:.3f} ms/step, "
        f"{flop / dt / 1e12:.1f} TFLOP/s, last loss {M.loss_dev.item():.3e}")


def converge_only(pk, h, sigma=2, d=2, iteration="ring", certificate="feasible"):
    """At (sigma, d, l = h): the plain FP64 iteration from zero, a certificate
    every TTB_CADENCE sweeps, until consecutive certificates move by less than
    1e-10 (B = the best bound then, also printed rounded down at the 6th
    decimal as the paper's tables print it); then, timed, plain FP64 from zero
    to B - 1e-9, and FP32 from zero + FP64 polish to B - 1e-9 in the same
    memory (the FP32 tables bound to the first halves of the FP64 tables'
    buffers, widened in place by the upcast).  Every run is one lcsb_run, on
    the ring or the two-array iteration, with Algorithm 2's or the largest-r
    certificate."""
    import torch
    P = new_ring(pk, sigma, d, h, "f64", iteration)
    log(f"plain FP64 {iteration} at sigma={sigma} d={d} l={h}: {P.n} indices, {P.stored} "
        f"stored, {P.nbuf * 8 * P.stored / 2**30:.0f} GiB of tables, branch means: {bool(P.means)}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.init_zero()
    cur, best, _, why = P.run(TTB_CADENCE, max_sweeps=MAX_SWEEPS, stop_delta=1e-10,
                              certificate=certificate)
    torch.cuda.synchronize()
    t_conv = time.perf_counter() - t0
    B = best["bound"]
    target = B - 1e-9
    log(f"converged: {B:.12f} after {cur['sweep']} sweeps, {t_conv:.2f} s ({why})")
    out = {"sigma": sigma, "d": d, "l": h, "indices": P.n, "stored": P.stored,
           "iteration": iteration, "certificate": certificate,
           "bound": B, "floor6": math.floor(B * 1e6) / 1e6,
           "converged_after_sweeps": cur["sweep"], "converged_after_s": round(t_conv, 3),
           "best_argmin_or_argmax": best["argmax_W"]}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.init_zero()
    cur, best, certs, _ = P.run(TTB_CADENCE, max_sweeps=MAX_SWEEPS, target=target,
                                certificate=certificate)
    torch.cuda.synchronize()
    out["plain_f64"] = {"seconds_to_target": round(time.perf_counter() - t0, 3),
                        "sweeps_to_target": cur["sweep"], "certificates": certs}
    log(f"plain to B - 1e-9: {out['plain_f64']['seconds_to_target']:.2f} s, {cur['sweep']} sweeps")
    M = new_ring(pk, sigma, d, h, "f32", iteration, bufs=[b.view(torch.float32) for b in P.bufs])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    M.init_zero()
    cur, best, certs32 = fp32_until_floor(M, certificate)
    sweeps32 = cur["sweep"]
    sweeps64, certs64, best = polish(P, M, best, target, certificate)
    torch.cuda.synchronize()
    t_mixed = time.perf_counter() - t0
    out["branch_means"] = {"f64": bool(P.means), "f32": bool(M.means)}
    out["mixed_f32_polish"] = {"seconds_to_target": round(t_mixed, 3), "sweeps_f32": sweeps32,
                               "sweeps_f64": sweeps64, "certificates": certs32 + certs64,
                               "bound": best["bound"], "reached": best["bound"] >= target}
    log(f"mixed to B - 1e-9: {t_mixed:.2f} s, {sweeps32} FP32 + {sweeps64} FP64 sweeps")
    print(json.dumps(out), flush=True)


def packed_only(pk, h):
    """sigma = d = 2 at l = h on exchange-packed tables (two-array iteration,
    largest-r certificate): plain FP64 from zero, a certificate every 16
    sweeps, until consecutive certificates move by less than 1e-10; then, in
    the same memory, FP32 from zero to its floor and the FP64 polish to that
    bound - 1e-9.  Prints one JSON line."""
    import torch
    torch.cuda.empty_cache()
    P = pk.Lcsb(2, 2, h, "f64", iteration="two_array_packed")
    log(f"packed FP64 pair at l={h}: {P.stored} entries per table, "
        f"{2 * P.stored * 8 / 2**30:.1f} GiB")
    stream = torch.cuda.current_stream()
    P.init_zero()
    P.iterate(2)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    e[0].record(stream)
    P.iterate(4)
    e[1].record(stream)
    e[2].record(stream)
    P.certify_optimal()
    e[3].record(stream)
    torch.cuda.synchronize()
    sweep_ms, cert_ms = e[0].elapsed_time(e[1]) / 4, e[2].elapsed_time(e[3])
    log(f"FP64 packed sweep {sweep_ms:.2f} ms, largest-r certificate {cert_ms:.2f} ms")
    t0 = time.perf_counter()
    P.init_zero()
    cur, best, certs, why = P.run(TTB_CADENCE, max_sweeps=MAX_SWEEPS, stop_delta=1e-10,
                                  certificate="optimal")
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    B = best["bound"]
    log(f"plain FP64: bound {B:.10f} after {cur['sweep']} sweeps ({why}), {t_plain:.1f} s")
    out = {"workload": f"sigma=2 d=2 l={h}: {4 ** h} tuples, exchange-packed "
                       f"({P.stored} entries per table), two-array iteration",
           "f64_sweep_ms": round(sweep_ms, 3), "f64_certificate_ms": round(cert_ms, 3),
           "plain_f64": {"bound": B, "sweeps": cur["sweep"], "certificates": certs,
                         "seconds": round(t_plain, 3), "stop": why,
                         "best_sweep": best["sweep"], "argmin": best["argmax_W"]}}
    M = pk.Lcsb(2, 2, h, "f32", iteration="two_array_packed",
                bufs=[b.view(torch.float32) for b in P.bufs])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    M.init_zero()
    cur, best32, certs32 = fp32_until_floor(M, "optimal")
    sweeps32 = cur["sweep"]
    sweeps64, certs64, best = polish(P, M, best32, B - 1e-9, "optimal")
    torch.cuda.synchronize()
    t_mixed = time.perf_counter() - t0
    log(f"FP32 floor {best32['bound']:.10f} after {sweeps32} sweeps; polished to "
        f"{best['bound']:.10f} after {sweeps64} FP64 sweeps, {t_mixed:.1f} s")
    out["mixed"] = {"fp32_floor_bound": best32["bound"], "sweeps_f32": sweeps32,
                    "sweeps_f64": sweeps64, "bound": best["bound"],
                    "reached": best["bound"] >= B - 1e-9, "seconds": round(t_mixed, 3),
                    "certificates": certs32 + certs64}
    print(json.dumps({"packed": out}), flush=True)


def two_array_f32_only(pk, h, max_sweeps, sigma=2, d=2):
    """The FP32 two-array iteration from zero at (sigma, d, l = h) with the
    largest-r certificate every TTB_CADENCE sweeps for max_sweeps sweeps (two
    FP32 tables: at l = 18, 2 x 128 GiB, the only form of the iteration that
    fits one GPU there).  Prints the best certified bound, rounded down at the
    6th decimal as the paper's tables print it, and the certificate trail."""
    import torch
    L = new_ring(pk, sigma, d, h, "f32", "two_array")
    log(f"two-array FP32 at sigma={sigma} d={d} l={h}: {L.n} indices, {L.stored} stored, "
        f"{2 * 4 * L.stored / 2**30:.0f} GiB, branch means: {bool(L.means)}")
    trail = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L.init_zero()
    best = None
    done = 0
    while done < max_sweeps:
        L.iterate(TTB_CADENCE)
        done += TTB_CADENCE
        cur, best = L.certify_optimal()
        trail.append((done, round(time.perf_counter() - t0, 3), cur["bound"], best["bound"]))
        log(f"sweep {done}: bound {cur['bound']:.10f} best {best['bound']:.10f} "
            f"rate {L.rate():.10f}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {"sigma": sigma, "d": d, "l": h, "indices": L.n, "stored": L.stored,
           "iteration": "two_array", "dtype": "f32", "sweeps": done, "seconds": round(dt, 3),
           "best_bound": best["bound"], "best_sweep": best["sweep"],
           "floor6": math.floor(best["bound"] * 1e6) / 1e6, "trail": trail}
    print(json.dumps(out), flush=True)


def certify_only(pk, h, sigma=2, d=2, dtype="f32"):
    """8 sweeps from zero at (sigma, d, l = h), then two certificates of each
    kind (Algorithm 2's, the largest-r one)."""
    import torch
    L = pk.Lcsb(sigma, d, h, dtype)
    L.init_zero()
    L.iterate(8)
    L.certify()
    L.certify()
    L.certify_optimal()
    L.certify_optimal()
    torch.cuda.synchronize()
    log(f"two certificates of each kind at sigma={sigma} d={d} l={h} {dtype}")


def copy_only(gib):
    """One plain device-to-device copy of `gib` GiB (after one warmup copy),
    the reference for scaling the HBM counters."""
    import torch
    n = int(gib * 2**30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    log(f"copied {n * 4} bytes twice")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(the library has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2407_10925_amd as pk

    torch.cuda.set_device(0)
    if args.profile_sweeps:
        return profile_only(pk, args.h, args.profile_sweeps, args.sigma, args.d, args.dtype,
                            not args.no_means)
    if args.copy_gib:
        return copy_only(args.copy_gib)
    if args.profile_seed:
        return seed_only(pk, args.h)
    if args.converge:
        return converge_only(pk, args.converge, args.sigma, args.d, args.iteration,
                             args.certificate)
    if args.profile_certify:
        return certify_only(pk, args.h, args.sigma, args.d, args.dtype)
    if args.two_array_f32:
        return two_array_f32_only(pk, args.two_array_f32, args.max_sweeps, args.sigma, args.d)
    if args.packed:
        return packed_only(pk, args.packed)
    if args.seed_ceiling:
        return seed_ceiling(pk, args.h, args.train_steps)
    if args.profile_train:
        return train_only(pk, args.h, args.profile_train, args.train_batch)
    if args.configs:
        return config_table(pk)
    h, cad = args.h, args.cadence
    n = 4 ** h
    L = pk.Lcsb(2, 2, h, "f32", means=True)
    stream = torch.cuda.current_stream()
    L.init_zero()
    log(f"warmup: {args.warmup} steps of {cad} sweeps + 1 certificate at l={h}")
    for _ in range(args.warmup):
        L.iterate(cad)
        L.certify_optimal()
    torch.cuda.synchronize()
    sweep_ms = []
    t0 = time.perf_counter()
    for s in range(args.steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        L.iterate(cad)
        e1.record(stream)
        cur, best = L.certify_optimal()
        sweep_ms.append(e0.elapsed_time(e1) / cad)
        log(f"step {s}: sweep {sweep_ms[-1]:.3f} ms, bound {cur['bound']:.9f}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    value = n * cad * args.steps / elapsed
    avg_sweep_s = statistics.mean(sweep_ms) * 1e-3
    algo_bytes = algorithmic_bytes(L, 4)
    folded = L.swap_symmetric()
    kernel = sweep_kernel(L, "float")
    achieved = algo_bytes / avg_sweep_s / 1e9
    computed = n // 4 + 2 ** (h - 1) if folded else n // 2
    traffic = measured_traffic()
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "kernel": kernel,
                "algorithmic_bytes_per_launch": algo_bytes,
                "avg_launch_ms": round(avg_sweep_s * 1e3, 4)}
    if traffic is not None:  # rocprofv3-measured HBM bytes per launch, at this launch time
        roofline["traffic_GBps"] = round(traffic / avg_sweep_s / 1e9, 1)
        roofline["traffic_frac"] = round(traffic / avg_sweep_s / 1e9 / HBM_PEAK_GBS, 4)
    del L
    torch.cuda.empty_cache()
    fp64 = fp64_sweep(pk, 14)
    log(f"plain FP64 sweep at l=14: {fp64['avg_launch_ms']} ms, {fp64['frac']} of peak")
    generality = config_table(pk, GENERALITY, emit=False)

    ttb = None
    if not args.no_ttb:
        ttb = time_to_bound(pk, h, args.train_steps)
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(pk, h, args.cpu_sample_log2)

    line = {
        "metric": METRIC, "value": value, "unit": "updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 sweeps, f64 certificate", "data": "synthetic (zero-start iteration)",
        "config": {"workload": f"sigma=2 d=2 l={h}: {n} table indices ({n // 2} stored, "
                               f"complement-folded; exchange-symmetric ring, one tuple of "
                               f"each exchanged pair computed and stored; branches read from the "
                               f"lags' branch-mean tables), FP32 renormalised sweeps, "
                               f"FP64 round-down largest-r certificate (one pass) every {cad} sweeps",
                   "sweeps_per_step": cad, "entries": n, "stored_entries": n // 2},
        "roofline": roofline,
        "fp64_sweep": fp64,
        # the other (sigma, d) shapes of the paper's Table 3 at their sizes:
        # sweep and certificate times, algorithmic bytes against the peak
        "configs": generality,
        "cpu_baseline": cpu,
        "time_to_bound": ttb,
        "sweep_only_updates_per_s": n / avg_sweep_s,
        # value counts every index of the table (n per sweep); the kernel
        # computes and stores one tuple of each orbit of the stored half under
        # the exchange of the strings (n / 4 pairs and 2^(l-1) fixed points),
        # which is what roofline.frac prices
        "computed_entries_per_sweep": computed,
        "computed_entries_per_s": computed * cad * args.steps / elapsed,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
