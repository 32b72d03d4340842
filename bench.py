"""Benchmark of the hot path on one MI355X.

One step = one exact distance computation of the throughput workload (an
additive code, n = 72 qubits, m = 72 i.i.d. Bernoulli(1/2) rows; seeded)
with every word of every codeword evaluated: input check, basis,
diagonalizations, planning, saved tables, every enumeration round and the
witness check, through the C ABI.  The step's input is a 10 KB host matrix;
the generator matrices the kernels read are built and kept in HBM by the
library inside the step.

Prints ONE JSON line:
  value        codewords/s over the timed steps: combinations enumerated by
               the rounds the exact distance needs, each codeword XORed and
               weighed in full, over wall time;
  time_to_exact_d_ms
               the same code on the library's default path (partial
               weights decide most codewords from their first word), timed
               over the same number of steps; its rate is reported as
               combinations certified per second, never as codewords/s;
  roofline     the enumeration kernel of the every-word run against the
               integer VALU peak, 4D+1 lane-ops per codeword (2D XOR, D OR,
               D popcount, 1 min), kernel time from HIP events recorded by
               the library on the launch stream;
  plain_per_code
               the plain per-round walk on the same code (one launch per
               (t, Gamma_j) round), the comparator of the engine;
  cpu_baseline the CPU oracle timed on the host's cores (single thread and
               all threads of the job's CPU share).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X vector ALU: 256 CUs x 128 32-bit lanes per clock x 2.4 GHz (the
# issue capacity behind the chip's 157.3 TFLOP/s fp32 vector figure: 4 SIMDs
# x 16 lanes x 2 VALU issues per cycle; single issue is half of it).
PEAK_LANE_OPS = 256 * 128 * 2.4e9
# MI355X dense fp4 (e2m1) MFMA peak, the published figure (no sparsity).
PEAK_FP4_FLOPS = 10.1e15


# HBM bytes per launch of the round kernel in the every-word run of this
# workload, from two rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE, each
# scaled by what it reads for a 1 GiB device copy in the same runs), valid
# only for the kernel source with this fingerprint (sha256 prefixes of
# round.hip and kernels.hpp, the enumeration kernel and its data layouts).
TRAFFIC = {"fingerprint": "82b3cf4ff46f732576d0919fb1fad4dc", "bytes_per_launch": 403461291}


def kernel_fingerprint():
    import hashlib
    out = ""
    for f in ("round.hip", "kernels.hpp"):
        with open(os.path.join(ROOT, "paper_2408_10743_amd", "csrc", f), "rb") as fh:
            out += hashlib.sha256(fh.read()).hexdigest()[:16]
    return out


def ops_per_codeword(D):
    """32-bit integer ops per codeword with every word evaluated: 2D XOR
    (x and z halves with the saved entry), D OR, D popcount and one MIN.
    The kernel fuses one XOR with the OR (v_bitop3), so it issues 3D + 1."""
    return 4 * D + 1


def issued_ops_per_codeword(D):
    return 3 * D + 1


def flops_per_codeword(n):
    """Matrix-core path: a codeword's weight is an affine function of the
    dot product of two sign vectors of length 3n (the x, z and x ^ z signs
    of every qubit), 3n multiply-adds."""
    return 2 * 3 * n


def mfma_flops_per_codeword(n):
    """What the MFMAs execute per codeword: K-steps of 128 signs, one per
    word (the last word packed into a spare group when it holds at most 10
    qubits)."""
    D = (n + 31) // 32
    ks = D - 1 if D >= 3 and n - 32 * (D - 1) <= 10 else D
    return 2 * 128 * ks


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1, help="GPUs (only 1 is supported)")
    ap.add_argument("--steps", type=int, default=10, help="timed calls on the main code")
    ap.add_argument("--warmup", type=int, default=2, help="untimed calls before them")
    ap.add_argument("--seed", type=int, default=0, help="seed of the main code (n = 72, m = 72)")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip timing the CPU oracle")
    ap.add_argument("--cpu-runs", type=int, default=5, help="runs of each CPU oracle sample (median reported)")
    ap.add_argument("--cpu-exact", action="store_true",
                    help="only time the CPU oracle's whole Brouwer-Zimmermann on the main code (3 runs), "
                         "its time to exact d")
    ap.add_argument("--no-extra", action="store_true", help="skip the batched, plain, serving and latency legs")
    ap.add_argument("--batch-codes", type=int, default=512, help="codes in the batched leg")
    ap.add_argument("--batch-max-work", type=float, default=1e11, help="largest predicted work of a batched code")
    ap.add_argument("--serve-requests", type=int, default=300, help="requests in the serving leg")
    ap.add_argument("--stab-codes", type=int, default=64, help="stabilizer codes in the modified-BZ leg")
    ap.add_argument("--serve-rate", type=float, default=0.0, help="requests/s (0: 60%% of measured capacity)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run 3 device copies of 1 GiB (reference for HBM byte counters)")
    ap.add_argument("--valu-probe", action="store_true",
                    help="only time the VALU instruction mixes of qd_valu_mix and print their rates")
    ap.add_argument("--default-only", action="store_true",
                    help="only run the default-path steps on the main code (partial weights), for a profiler")
    ap.add_argument("--vector-alu", action="store_true",
                    help="with --every-word-only or --default-only: the vector-ALU kernels (matrix_cores -1)")
    ap.add_argument("--every-word-only", action="store_true",
                    help="only run the timed steps on the main code (every word evaluated) and print their "
                         "rate and roofline, for a profiler")
    ap.add_argument("--walk-only", action="store_true",
                    help="only run the plain per-round walk on the same code (--steps timed calls after "
                         "one warm-up call), for a profiler")
    ap.add_argument("--batch-only", action="store_true",
                    help="only run the config-4 batch leg (two batched calls and the per-code loop), for a profiler")
    ap.add_argument("--first-draws-only", action="store_true",
                    help="only run the unfiltered config-4 draws (first --batch-codes draws, per-code budget)")
    ap.add_argument("--tune-out", default="",
                    help="only run the launch-shape tuner (qd_tune_run, up to 300 s) and write its table to this file")
    ap.add_argument("--serving-only", action="store_true",
                    help="only run the two serving legs (default path and every word) and print them")
    ap.add_argument("--latency-only", action="store_true",
                    help="only run the time-to-exact-d leg on configs 1 and 2, for a profiler")
    ap.add_argument("--round-sweep", action="store_true",
                    help="only run one large round (48 two-row packages, t = 6) at D = 1..4 words per "
                         "half, for per-D kernel durations from a profiler")
    return ap.parse_args()


def cpu_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    affinity = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    omp = os.environ.get("OMP_NUM_THREADS")
    return {"model": model, "nproc": os.cpu_count(), "affinity": affinity,
            "OMP_NUM_THREADS": int(omp) if omp and omp.isdigit() else None}


def oracle_exact_combinations(seed):
    """Combinations the oracle's BZ enumerates on config 3 to reach the exact
    distance, from its recorded trace (written by tests/golden/make_golden.py,
    which calls only the oracle); None when the trace was not recorded."""
    path = os.path.join(ROOT, "tests", "golden", "oracle_distances.json")
    try:
        rounds = json.load(open(path))["config3_oracle_rounds"][seed]
    except (OSError, KeyError, IndexError):
        return None
    return sum(r[4] for r in rounds)


def cpu_baseline(G, field, runs, seed):
    """The oracle's plain enumeration of the same code's rounds, built -O3
    -march=native on this host: rounds t = 1..5 of both generator matrices
    on one thread (1.8e8 codewords) and t = 1..6 on all threads of the
    job's CPU share (2.9e9 codewords), `runs` runs each, medians.  The
    oracle's time to exact d is extrapolated from the all-thread rate and
    the combinations its BZ enumerates (recorded trace)."""
    from oracle import oracle as O
    O.use_native()
    info = cpu_info()
    threads = min(info["affinity"], info["OMP_NUM_THREADS"] or info["affinity"])
    B = O.expand(G, field)
    gs = O.gamma(B, O.DIAG_F4, 2, with_rows=True)

    def sample(tmax, nthreads):
        rates, visited = [], 0
        for _ in range(runs):
            visited, wall = 0, 0.0
            for t in range(1, tmax + 1):
                for g in gs:
                    t0 = time.perf_counter()
                    _, _, cnt = O.round_min(g["rows"], g["dims"], t, nthreads=nthreads)
                    wall += time.perf_counter() - t0
                    visited += cnt
            rates.append(visited / wall)
        rates.sort()
        return rates[len(rates) // 2], visited, rates

    r1, v1, all1 = sample(5, 1)
    rn, vn, alln = sample(6, threads)
    exact = oracle_exact_combinations(seed)
    out = {"value": rn, "unit": "codewords/s", "cores": threads, "kind": "oracle",
           "sample": f"oracle (gcc -O3 -march=native, OpenMP) plain enumeration of the same code: rounds t=1..6 of "
                     f"both generator matrices ({vn} codewords) on {threads} threads, median of {runs} runs; "
                     f"single thread: rounds t=1..5 ({v1} codewords), median of {runs} runs",
           "single_thread_codewords_per_s": r1, "all_threads_codewords_per_s": rn,
           "runs_single": all1, "runs_all": alln, "cpu": info,
           "build": "gcc -O3 -march=native -fopenmp"}
    if exact is not None:
        out["oracle_exact_d_combinations"] = exact
        out["time_to_exact_d_s_extrapolated"] = exact / rn
        out["time_to_exact_d_s_single_thread_extrapolated"] = exact / r1
    return out


def cpu_exact(G, field, seed, runs=3):
    """The oracle's whole Brouwer-Zimmermann on the main code, -O3
    -march=native, all threads of the job's CPU share: time to exact d."""
    from oracle import oracle as O
    O.use_native()
    info = cpu_info()
    threads = min(info["affinity"], info["OMP_NUM_THREADS"] or info["affinity"])
    B = O.expand(G, field)
    ts, d, combos = [], None, 0
    for i in range(runs):
        t0 = time.perf_counter()
        d, _, log = O.bz(B, O.DIAG_F4, 2, nthreads=threads)
        ts.append(time.perf_counter() - t0)
        combos = sum(r[4] for r in log)
        print(f"oracle BZ run {i}: d={d} {ts[-1]:.2f} s", file=sys.stderr, flush=True)
    ts.sort()
    return {"d": d, "median_s": ts[len(ts) // 2], "runs_s": ts, "combinations": combos,
            "codewords_per_s": combos / ts[len(ts) // 2], "threads": threads, "cpu": info, "seed": seed}


def predicted_work(Q, G, f):
    """Planner-predicted combinations of the cheaper of the F2 and F4
    constructions, enumerating every codeword.  This defines which draws
    the workloads keep, so it counts all three codewords of each F4 scalar
    class even though the library enumerates one of them."""
    p = Q.qd_plan(G, f)
    f4 = p["predicted_f4"] * (3 if p["f4_scalar_classes"] else 1)
    cands = [x for x in (p["predicted_f2"], f4) if x >= 0]
    return min(cands)


def config4_codes(Q, W, count, max_work):
    """Draws config-4 codes in order and keeps the first `count` whose
    planner-predicted work is at most max_work (the stated distribution has
    a tail far beyond any budget: 1e13..1e17 codewords)."""
    kept, drawn = [], 0
    pool = W.config4(count * 8)
    for G, f in pool:
        drawn += 1
        if predicted_work(Q, G, f) <= max_work:
            kept.append((G, f))
            if len(kept) == count:
                break
    return kept, drawn


def kernel_roofline(stats, launches=None):
    """Roofline of the enumeration kernel over runs with every word
    evaluated: codewords the kernel enumerated (rounds run ahead included)
    x the work per codeword, over the kernel time spent on them (HIP events
    on the launch stream, shared among a launch's codes by their tiles).
    On the matrix cores the work is 6n flops (3n sign multiply-adds)
    against the fp4 MFMA peak; on the vector ALU (4D+1) lane-ops against
    the lane-op peak."""
    ms = sum(s.enumerated_kernel_ms for s in stats)
    assert all(s.words == s.D * s.enumerated for s in stats), "not an every-word run"
    enumerated = sum(s.enumerated for s in stats)
    mc = [s for s in stats if s.matrix_core_launches == s.launches and s.launches > 0]
    va = [s for s in stats if s.matrix_core_launches == 0]
    if mc and len(mc) < len(stats):
        # A batch of both kinds (one-word codes and small rounds keep the vector
        # ALU): each part against its own peak; codes whose launches were of
        # both kinds are left out of both.
        out = {"bound": "mixed", "frac": None, "codewords_enumerated": enumerated, "kernel_ms_total": ms,
               "matrix_cores": kernel_roofline(mc), "codes_matrix_cores": len(mc),
               "codes_vector_alu": len(va), "codes_both": len(stats) - len(mc) - len(va)}
        if va:
            out["vector_alu"] = kernel_roofline(va)
        return out
    if mc:
        flops = sum(s.enumerated * flops_per_codeword(s.n) for s in stats)
        hw = sum(s.enumerated * mfma_flops_per_codeword(s.n) for s in stats)
        achieved = flops / (ms * 1e-3)
        out = {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_FP4_FLOPS / 1e12, "unit": "TFLOP/s",
               "frac": achieved / PEAK_FP4_FLOPS,
               "ops_basis": "6n flops per codeword: the 3n-sign dot product (x, z, x^z signs per qubit), "
                            "fp4 e2m1 operands, fp32 sums, exact",
               "codewords_enumerated": enumerated, "kernel_ms_total": ms,
               "frac_executed": hw / (ms * 1e-3) / PEAK_FP4_FLOPS}
    else:
        ops = sum(s.enumerated * ops_per_codeword(s.D) for s in stats)
        issued = sum(s.enumerated * issued_ops_per_codeword(s.D) for s in stats)
        achieved = ops / (ms * 1e-3)
        out = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12, "unit": "TOP/s",
               "frac": achieved / PEAK_LANE_OPS,
               "ops_basis": "4D+1 lane-ops per codeword (2D XOR, D OR, D popcount, 1 min)",
               "codewords_enumerated": enumerated, "kernel_ms_total": ms,
               "frac_issued_3D1": issued / (ms * 1e-3) / PEAK_LANE_OPS}
    if launches:
        out["launches"] = launches
        out["avg_launch_ms"] = ms / launches
        out["codewords_per_launch"] = out["codewords_enumerated"] / launches
    return out


def run_batch(Q, codes, budget, **opts):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, ds, wits, sts, stats = Q.qd_distance_batch(codes, budget=budget, **opts)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, ds, sts, stats


def leg_batched(Q, W, a):
    """Config 4 (the kept draws): the batch to exact d on the default path
    against a loop of per-code calls, and the same batch with every word
    evaluated for codewords/s and the kernel's roofline."""
    codes, drawn = config4_codes(Q, W, a.batch_codes, a.batch_max_work)
    budget = int(a.batch_max_work * 4)
    # The first call also fills the library's device-memory pool (tables of
    # every code); the timed calls come after it, as the per-code loop below
    # runs with a warm pool too.
    t_cold, _, _, _ = run_batch(Q, codes, budget)
    runs = [run_batch(Q, codes, budget) for _ in range(3)]
    runs.sort(key=lambda r: r[0])
    t_batch, ds, sts, stats = runs[1]
    comb_b = sum(s.combinations for s in stats)
    words_b = sum(s.words for s in stats)
    enum_b = sum(s.enumerated for s in stats)
    t0 = time.perf_counter()
    comb_p, ds_p, kms_p = 0, [], 0.0
    for G, f in codes:
        st1, d1, _, s1 = Q.qd_distance_ex(G, f, budget=budget, timing=1)
        comb_p += s1.combinations
        kms_p += s1.kernel_ms
        ds_p.append(d1)
    t_plain = time.perf_counter() - t0
    # every word evaluated (codewords/s and roofline); timing on
    run_batch(Q, codes, budget, partial_weight=-1)
    fw = [run_batch(Q, codes, budget, partial_weight=-1, timing=1) for _ in range(3)]
    fw.sort(key=lambda r: r[0])
    t_fw, ds_fw, sts_fw, stats_fw = fw[1]
    comb_fw = sum(s.combinations for s in stats_fw)
    _, _, _, stats_bt = run_batch(Q, codes, budget, timing=1)
    # The same batch under the fixed launch-shape rules (no tuning table).
    st_t, tuned = Q.qd_tune_get()
    n_tuned = len(json.loads(tuned)["entries"]) if st_t == 0 else 0
    t_rules = None
    if n_tuned:
        Q.qd_tune_reset()
        run_batch(Q, codes, budget)
        rr = sorted(run_batch(Q, codes, budget)[0] for _ in range(3))
        t_rules = rr[1]
        Q.qd_tune_load(tuned)
    ns = [G.shape[1] // 2 if f == 2 else G.shape[1] for G, f in codes]
    return {
        "workload": f"config 4: first {len(codes)} of {drawn} drawn codes (n~U{{24..96}}, even additive m~U{{n-8..n+8}}, "
                    f"odd F4-linear k=n/2) with planner-predicted work <= {a.batch_max_work:.0e}; budget {budget:.0e}",
        "codes": len(codes), "drawn": drawn, "n_range": [min(ns), max(ns)],
        "exact": sum(1 for x in sts if x == 0), "incomplete": sum(1 for x in sts if x == 1),
        "same_d_as_per_code": ds == ds_p, "same_d_every_word": ds_fw == ds,
        "time_to_exact_d_s": t_batch, "batched_first_call_s": t_cold,
        "per_code_loop_s": t_plain, "speedup_vs_per_code_loop": t_plain / t_batch,
        "tuned_buckets": n_tuned, "time_to_exact_d_s_fixed_rules": t_rules,
        "per_code_loop_kernel_s": kms_p * 1e-3,
        "batched_kernel_s": sum(s.kernel_ms for s in stats_bt) * 1e-3,
        "combinations_certified_per_s": comb_b / t_batch,
        "words_per_codeword": words_b / max(enum_b, 1),
        "every_word": {"time_s": t_fw, "codewords_per_s": comb_fw / t_fw,
                       "roofline": kernel_roofline(stats_fw)},
    }


def leg_first_draws(Q, W, a):
    """Config 4 as drawn, without the work filter: the first 512 draws (n up
    to 96, both fields) in one batch with the same per-code budget.  Codes
    whose certified bounds do not meet within the budget end as
    QD_INCOMPLETE with [L, U]; they are reported apart and excluded from the
    exactness claims."""
    codes = W.config4(a.batch_codes)
    budget = int(a.batch_max_work * 4)
    t_batch, ds, sts, stats = run_batch(Q, codes, budget)
    ns = [G.shape[1] // 2 if f == 2 else G.shape[1] for G, f in codes]
    inc = [{"draw": i, "n": ns[i], "field": codes[i][1], "m": int(codes[i][0].shape[0]),
            "L": stats[i].L, "U": stats[i].U, "combinations": stats[i].combinations}
           for i in range(len(codes)) if sts[i] == 1]
    exact = [i for i in range(len(codes)) if sts[i] == 0]
    big = [i for i in range(len(codes)) if ns[i] >= 81]
    return {"workload": f"config 4 as drawn: the first {len(codes)} draws, no work filter, budget {budget:.0e} "
                        f"combinations per code",
            "codes": len(codes), "n_range": [min(ns), max(ns)], "time_s": t_batch,
            "exact": len(exact), "incomplete": len(inc), "errors": sum(1 for x in sts if x < 0),
            "n_81_96": {"codes": len(big), "exact": sum(1 for i in big if sts[i] == 0)},
            "exact_n_range": [min(ns[i] for i in exact), max(ns[i] for i in exact)] if exact else None,
            "combinations": sum(s.combinations for s in stats),
            "incomplete_bounds": inc}


def leg_unrank(Q, G, field, engine_step_ms):
    """A per-code path without saved sums or a walk: every lane unranks and
    XORs its whole combination (t rows per codeword)."""
    st, d, wit, s = Q.qd_distance_ex(G, field, saved_depth=-1, tops_mode=2, timing=1)
    assert st == 0
    return {"ms_per_step": s.wall_ms, "codewords_per_s": s.combinations / (s.wall_ms * 1e-3),
            "kernel_codewords_per_s": s.combinations / (s.kernel_ms * 1e-3), "d": d,
            "engine_speedup": s.wall_ms / engine_step_ms}


def leg_walk(Q, G, field, stream, engine_step_ms, steps):
    """The plain per-round walk on the same code (qd_options.walk = 1): one
    launch per (t, Gamma_j) round and a readback of U after each; lanes walk
    package sets in revolving-door order and element choices in reflected
    ternary Gray order, every codeword evaluated in full.  One warm-up call,
    then `steps` timed calls."""
    runs = []
    for i in range(steps + 1):
        st, d, wit, s = Q.qd_distance_ex(G, field, stream=stream, timing=1, walk=1)
        assert st == 0
        if i:
            runs.append(s)
    combos = sum(s.combinations for s in runs)
    walked = sum(s.words for s in runs) / runs[0].D  # codewords evaluated
    kernel_ms = sum(s.kernel_ms for s in runs)
    wall_ms = sum(s.wall_ms for s in runs)
    D = runs[0].D
    ms = wall_ms / steps
    return {"kind": "plain per-round walk: one launch per (t, Gamma_j), revolving-door package sets x "
                    "ternary Gray element choices, every word of every codeword evaluated",
            "d": d, "ms_per_step": ms, "codewords_per_s": combos / (wall_ms * 1e-3),
            "kernel_codewords_per_s": combos / (kernel_ms * 1e-3),
            "walked_per_combination": walked / combos,
            "launches_per_step": sum(s.launches for s in runs) / steps,
            # per walked codeword: 2D XOR + D OR + D v_bcnt + 1 min
            "roofline_frac": walked * ops_per_codeword(D) / (kernel_ms * 1e-3) / PEAK_LANE_OPS,
            "engine_speedup": ms / engine_step_ms,
            "target_5x_engine_ms": ms / 5}


def leg_constructions(Q, W):
    """Time to exact d per construction -- the paper's Saved_1_Gamma (F2),
    Saved_2_Gamma generalized (F4) and Saved_isometry -- on config 2 seeds
    0..4 and config 3 seed 0; a construction is skipped where its planned
    work exceeds 1e12 combinations."""
    out = {}
    for name, cases in (("config2", [W.config2(i) for i in range(5)]), ("config3", [W.config3(0)])):
        res = {}
        for label, diag in (("F2", Q.QD_DIAG_F2), ("F4", Q.QD_DIAG_F4), ("isometry", Q.QD_DIAG_ISO)):
            if any(Q.qd_plan(G, f, diag)["predicted_" + ("iso" if diag == Q.QD_DIAG_ISO else label.lower())] > 1e12
                   for G, f in cases):
                res[label] = "skipped (planned work > 1e12)"
                continue
            ms, comb, ds = [], 0, []
            for G, f in cases:
                Q.qd_distance_ex(G, f, diag=diag)
                t0 = time.perf_counter()
                st, d, _, s = Q.qd_distance_ex(G, f, diag=diag)
                ms.append((time.perf_counter() - t0) * 1e3)
                assert st == 0
                comb += s.combinations
                ds.append(d)
            res[label] = {"mean_ms": sum(ms) / len(ms), "codewords": comb, "d": ds}
        out[name] = res
    return out


def leg_stabilizer(Q, W, a):
    """Quantum stabilizer codes shaped like the paper's larger data set
    (normalizer matrices, n 32..64, K/N 0.586..0.758), distance with the
    Modified-BZ filter: a batch of the first draws whose predicted work is
    at most --batch-max-work, and each construction timed alone on the
    first four of them."""
    codes, drawn, i = [], 0, 0
    while len(codes) < a.stab_codes and drawn < 20 * a.stab_codes:
        A, f = W.config_stab(i)
        i += 1
        drawn += 1
        if predicted_work(Q, A, f) <= a.batch_max_work:
            codes.append((A, f))
    flt = Q.QD_FILTER_STABILIZER
    t0 = time.perf_counter()
    st, ds, _, sts, stats = Q.qd_distance_batch(codes, filter=flt, budget=int(a.batch_max_work * 4))
    t_batch = time.perf_counter() - t0
    comb = sum(s.combinations for s in stats)
    diags = {}
    for s in stats:
        diags[{2: "F2", 3: "isometry", 4: "F4"}[s.diag]] = diags.get({2: "F2", 3: "isometry", 4: "F4"}[s.diag], 0) + 1
    per = {}
    for label, diag in (("F2", Q.QD_DIAG_F2), ("F4", Q.QD_DIAG_F4), ("isometry", Q.QD_DIAG_ISO)):
        ms, skip = [], False
        for A, f in codes[:4]:
            p = Q.qd_plan(A, f, diag)
            if p["predicted_" + {2: "f2", 3: "iso", 4: "f4"}[diag]] > 1e12:
                skip = True
                break
            Q.qd_distance_ex(A, f, diag=diag, filter=flt)
            t1 = time.perf_counter()
            Q.qd_distance_ex(A, f, diag=diag, filter=flt)
            ms.append((time.perf_counter() - t1) * 1e3)
        per[label] = "skipped (planned work > 1e12)" if skip else {"mean_ms": sum(ms) / len(ms)}
    ns = [A.shape[1] // 2 for A, _ in codes]
    ks = [A.shape[0] - A.shape[1] // 2 for A, _ in codes]
    return {"workload": f"{len(codes)} of {drawn} random [[n,k]] stabilizer codes, n {min(ns)}..{max(ns)}, "
                        f"k {min(ks)}..{max(ks)}, predicted work <= {a.batch_max_work:.0e}",
            "exact": sum(1 for x in sts if x == 0), "d_range": [min(ds), max(ds)],
            "batched_s": t_batch, "codewords_per_s": comb / t_batch, "constructions_chosen": diags,
            "first4_time_to_exact_d": per}


def leg_latency(Q, W):
    out = {}
    for name, fn in (("config1", W.config1), ("config2", W.config2)):
        ts = []
        for i in range(10):
            G, f = fn(i)
            Q.qd_distance(G, f)
            t0 = time.perf_counter()
            st, d, _ = Q.qd_distance(G, f)
            ts.append((time.perf_counter() - t0) * 1e3)
        ts.sort()
        out[name] = {"median_ms": ts[len(ts) // 2], "max_ms": ts[-1], "codes": len(ts)}
    return out


def serving_requests(Q, W, a):
    raw = W.config5(a.serve_requests * 4, 1.0)
    reqs, drawn = [], 0
    for _, G, f in raw:
        drawn += 1
        if predicted_work(Q, G, f) <= 1e10:
            reqs.append((G, f))
            if len(reqs) == a.serve_requests:
                break
    return reqs, drawn


def leg_serving(Q, W, a, **opts):
    """Config 5: Poisson arrivals, n log-uniform in 16..96, alternately
    additive (m = n) and F4-linear (k = n/2); requests whose predicted work
    exceeds 1e10 are redrawn (stated in the output).  opts apply to every
    request (partial_weight=-1: every word evaluated)."""
    reqs, drawn = serving_requests(Q, W, a)

    def back_to_back():
        """Service capacity: the serving engine given every request at once."""
        e = Q.qd_engine_create()
        t0 = time.perf_counter()
        for i, (G, f) in enumerate(reqs):
            Q.qd_engine_submit(e, G, f, i, **opts)
        done = 0
        while done < len(reqs):
            done += len(Q.qd_engine_poll(e, 64, 100))
        t = time.perf_counter() - t0
        Q.qd_engine_destroy(e)
        return t

    back_to_back()  # device memory and tables warm
    t_all = back_to_back()
    rate = a.serve_rate or 0.6 * len(reqs) / t_all
    gaps = [t for t, _, _ in W.config5(len(reqs), rate, index=1)]
    e = Q.qd_engine_create()
    lat, comb, statuses = [], 0, []
    t_start = time.perf_counter()
    for i, (G, f) in enumerate(reqs):
        while time.perf_counter() - t_start < gaps[i]:
            for r, w in Q.qd_engine_poll(e, 64, 0):
                lat.append(r.latency_ms); comb += r.combinations; statuses.append(r.status)
            time.sleep(0.0002)
        Q.qd_engine_submit(e, G, f, i, **opts)
    while len(lat) < len(reqs):
        for r, w in Q.qd_engine_poll(e, 64, 100):
            lat.append(r.latency_ms); comb += r.combinations; statuses.append(r.status)
    t_total = time.perf_counter() - t_start
    Q.qd_engine_destroy(e)
    lat.sort()
    key = "codewords_per_s" if opts.get("partial_weight") == -1 else "combinations_certified_per_s"
    return {"workload": f"config 5: {len(reqs)} requests of {drawn} drawn (predicted work <= 1e10), "
                        f"Poisson rate {rate:.1f}/s (60% of the engine's back-to-back capacity)",
            "rate_per_s": rate, "requests": len(reqs), "exact": sum(1 for x in statuses if x == 0),
            "p50_ms": lat[len(lat) // 2], "p99_ms": lat[min(len(lat) - 1, int(0.99 * len(lat)))],
            key: comb / t_total, "window_s": t_total}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the enumeration of one code "
              f"shards by rank ranges, which this library does not run across GPUs.", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2408_10743_amd import qdist as Q
    from paper_2408_10743_amd import workloads as W

    torch.cuda.set_device(0)
    st, name = Q.qd_device_check()
    if st != 0:
        print(f"device check failed: {Q.qd_strerror(st)} ({name})", file=sys.stderr)
        sys.exit(1)
    if a.round_sweep:
        out = {}
        for D in (1, 2, 3, 4):
            n = 32 * D
            rows, dims = W.random_packages(48, n, W.config_seed(50, D), 1.0)
            for rep in range(2):  # the second call's kernel is the one to read
                t0 = time.perf_counter()
                st, wmin, _, count = Q.qd_round_min(rows, dims, 6)
                ms = (time.perf_counter() - t0) * 1e3
                if st != 0:
                    raise RuntimeError(Q.qd_strerror(st))
            out[f"D{D}"] = {"n": n, "combinations": count, "ops_per_codeword": ops_per_codeword(D),
                            "wall_ms": ms, "wmin": wmin}
        print(json.dumps({"round_sweep": out}))
        return
    if a.valu_probe:
        rates = {}
        for name_, mix in Q.QD_MIXES.items():
            st, v = Q.qd_valu_mix(mix)
            if st != 0:
                raise RuntimeError(Q.qd_strerror(st))
            rates[name_] = v
        print(json.dumps({"valu_mix_lane_ops_per_s": rates, "peak_lane_ops_per_s": PEAK_LANE_OPS}))
        return
    stream = torch.cuda.current_stream()
    G, field = W.config3(a.seed)
    if a.tune_out:
        t0 = time.perf_counter()
        st, text = Q.qd_tune_run(300.0)
        if st not in (0, Q.QD_INCOMPLETE):
            raise RuntimeError(Q.qd_strerror(st))
        with open(a.tune_out, "w") as fh:
            fh.write(text)
        print(json.dumps({"tune": {"status": st, "seconds": time.perf_counter() - t0,
                                   "entries": len(json.loads(text)["entries"]), "file": a.tune_out}}))
        return
    if a.cpu_exact:
        print(json.dumps({"cpu_exact": cpu_exact(G, field, a.seed)}))
        return
    if a.batch_only:
        print(json.dumps({"batched": leg_batched(Q, W, a)}))
        return
    if a.first_draws_only:
        print(json.dumps({"batched_first_draws": leg_first_draws(Q, W, a)}))
        return
    if a.latency_only:
        print(json.dumps({"latency": leg_latency(Q, W)}))
        return
    if a.serving_only:
        print(json.dumps({"serving": leg_serving(Q, W, a),
                          "serving_every_word": leg_serving(Q, W, a, partial_weight=-1)}))
        return
    if a.walk_only:
        print(json.dumps({"walk_per_round": leg_walk(Q, G, field, stream.cuda_stream, float("nan"), a.steps)}))
        return

    def run(steps, **opts):
        """`steps` calls on the main code, bracketed by device syncs (each call
        returns after its device work, so s.wall_ms times one call)."""
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = []
        for _ in range(steps):
            st, d, wit, s = Q.qd_distance_ex(G, field, stream=stream.cuda_stream, timing=1, **opts)
            if st != 0:
                raise RuntimeError(Q.qd_strerror(st))
            out.append((d, s))
        torch.cuda.synchronize()
        return time.perf_counter() - t0, out

    def median_ms(stats):
        w = sorted(s.wall_ms for _, s in stats)
        return w[len(w) // 2]

    kopt = {"matrix_cores": -1} if a.vector_alu else {}
    if a.default_only:
        run(a.warmup, **kopt)
        wall, stats = run(a.steps, **kopt)
        print(json.dumps({"default_path_ms_per_step": wall * 1e3 / a.steps}))
        return
    def copy_calibration():
        """Three device copies of 1 GiB: the reference for HBM byte counters."""
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        return src.numel() * 4

    if a.every_word_only:
        run(a.warmup, partial_weight=-1, **kopt)
        wall, stats = run(a.steps, partial_weight=-1, **kopt)
        roof = kernel_roofline([s for _, s in stats], sum(s.launches for _, s in stats))
        out = {"ms_per_step": wall * 1e3 / a.steps,
               "codewords_per_s": sum(s.combinations for _, s in stats) / wall, "roofline": roof}
        if a.copy_calibration:
            out["copy_calibration_bytes"] = copy_calibration()
        print(json.dumps(out))
        return

    # The step: every word of every codeword evaluated (partial_weight -1).
    run(a.warmup, partial_weight=-1)
    wall, stats = run(a.steps, partial_weight=-1)
    d = stats[0][0]
    assert all(x[0] == d for x in stats)
    combos = sum(s.combinations for _, s in stats)
    kernel_ms = sum(s.kernel_ms for _, s in stats)
    launches = sum(s.launches for _, s in stats)
    D = stats[0][1].D
    s0 = stats[0][1]
    roof = kernel_roofline([s for _, s in stats], launches)
    roof["kernel"] = (f"qd_round_kernel<{D}, false, every word on the matrix cores>" if roof["bound"] == "mfma"
                      else f"qd_round_kernel<{D}, false, every word>")
    roof["traffic"] = TRAFFIC["bytes_per_launch"] if kernel_fingerprint() == TRAFFIC["fingerprint"] else None
    # The library's default path on the same code: time to exact d.
    run(a.warmup)
    wall_d, stats_d = run(a.steps)
    assert all(x[0] == d for x in stats_d)
    combos_d = sum(s.combinations for _, s in stats_d)
    words_d = sum(s.words for _, s in stats_d)
    enum_d = sum(s.enumerated for _, s in stats_d)
    ttd_ms = wall_d * 1e3 / a.steps
    # The same two legs on the vector-ALU kernels (qd_options.matrix_cores -1).
    vsteps = max(1, min(a.steps, 5))
    run(1, partial_weight=-1, matrix_cores=-1)
    wall_v, stats_v = run(vsteps, partial_weight=-1, matrix_cores=-1)
    run(1, matrix_cores=-1)
    wall_vd, stats_vd = run(vsteps, matrix_cores=-1)
    assert all(x[0] == d for x in stats_v + stats_vd)
    vector_alu = {
        "kind": "the same code on the vector-ALU kernels (matrix_cores -1)",
        "ms_per_step": wall_v * 1e3 / vsteps,
        "codewords_per_s": sum(s.combinations for _, s in stats_v) / wall_v,
        "time_to_exact_d_ms": wall_vd * 1e3 / vsteps,
        "roofline": kernel_roofline([s for _, s in stats_v], sum(s.launches for _, s in stats_v)),
    }
    out = {
        "metric": "codewords/s (XOR+symplectic wt) & time-to-exact-d: batched vs plain per-code",
        "value": combos / wall,
        "unit": "codewords/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": wall * 1e3 / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp4" if roof["bound"] == "mfma" else "u32",
        "data": "synthetic",
        "config": {"workload": f"single additive code n=72 m=72 Bernoulli(1/2), seed {a.seed} (config 3), "
                               f"exact d with every word of every codeword evaluated",
                   "d": d, "diag": "F4" if s0.diag == 4 else "F2", "gammas": s0.h,
                   "packages": list(s0.P)[:s0.h], "delta": list(s0.delta)[:s0.h],
                   "rounds": s0.nlog, "codewords_per_step": combos // a.steps},
        "kernel_codewords_per_s": combos / (kernel_ms * 1e-3),
        "median_ms_per_step": median_ms(stats),
        "host_ms_per_step": sum(s.host_ms for _, s in stats) / a.steps,
        "time_to_exact_d_ms": ttd_ms,
        "time_to_exact_d_ms_median": median_ms(stats_d),
        "default_path": {
            "kind": "the library's default path: partial weights decide a codeword from its first words "
                    "plus a pivot credit, completing only blocks that may hold a weight below U",
            "time_to_exact_d_ms": ttd_ms,
            "combinations_certified_per_s": combos_d / wall_d,
            "words_per_codeword": words_d / enum_d,
            "kernel_ms_per_step": sum(s.kernel_ms for _, s in stats_d) / a.steps,
            "speedup_vs_every_word": (wall * 1e3 / a.steps) / ttd_ms,
        },
        "roofline": roof,
        "vector_alu": vector_alu,
        "device": name,
    }
    if a.copy_calibration:
        out["copy_calibration_bytes"] = copy_calibration()
    if not a.no_extra:
        out["plain_per_code"] = leg_walk(Q, G, field, stream.cuda_stream, ttd_ms, 3)
        out["plain_per_code"]["engine_every_word_speedup"] = out["plain_per_code"]["ms_per_step"] / out["ms_per_step"]
        out["unrank_per_lane"] = leg_unrank(Q, G, field, ttd_ms)
        out["batched"] = leg_batched(Q, W, a)
        out["batched_first_draws"] = leg_first_draws(Q, W, a)
        out["serving"] = leg_serving(Q, W, a)
        out["serving_every_word"] = leg_serving(Q, W, a, partial_weight=-1)
        out["latency"] = leg_latency(Q, W)
        out["constructions"] = leg_constructions(Q, W)
        out["stabilizer"] = leg_stabilizer(Q, W, a)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(G, field, a.cpu_runs, a.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
