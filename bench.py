"""Benchmark of the hot path on one MI355X.

One step = one exact distance computation of the throughput workload (an
additive code, n = 72 qubits, m = 72 i.i.d. Bernoulli(1/2) rows; seeded):
input check, basis, diagonalizations, planning, saved tables, every
enumeration round and the witness check, through the C ABI.  The step's
input is a 10 KB host matrix; the generator matrices the kernels read are
built and kept in HBM by the library inside the step.

Prints ONE JSON line: codewords/s over the timed steps (combinations
actually visited / wall time), the time to an exact d, the roofline of the
enumeration kernel (integer VALU bound) measured with HIP events on the
launch stream, and the CPU oracle timed on a bounded sample of the same
workload.
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


# HBM bytes per launch of the round kernel on this workload, from two
# rocprofv3 --pmc passes (FETCH_SIZE x2.0, WRITE_SIZE x1.0, factors from a
# 1 GiB device copy in the same runs), valid only for the kernel source
# with this fingerprint (sha256 prefixes of round.hip and kernels.hpp, the
# enumeration kernel and its data layouts).
TRAFFIC = {"fingerprint": "d01b1ee72cb9aa6e210d0fd35c79cca9", "bytes_per_launch": 836256280}


def kernel_fingerprint():
    import hashlib
    out = ""
    for f in ("round.hip", "kernels.hpp"):
        with open(os.path.join(ROOT, "paper_2408_10743_amd", "csrc", f), "rb") as fh:
            out += hashlib.sha256(fh.read()).hexdigest()[:16]
    return out


def ops_per_codeword(D):
    """32-bit integer ops per codeword with every word evaluated: per word
    one XOR (x), one fused XOR-OR (z, v_bitop3) and one popcount, plus one
    MIN."""
    return 3 * D + 1


def algorithmic_ops(words, combos):
    """Integer ops the enumeration needs: three per evaluated word and one
    MIN per codeword.  With partial weights a codeword whose first words
    already decide it costs fewer words; without, words = D x combos and
    this is combos x ops_per_codeword(D)."""
    return 3 * words + combos


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1, help="GPUs (only 1 is supported)")
    ap.add_argument("--steps", type=int, default=10, help="timed calls on the main code")
    ap.add_argument("--warmup", type=int, default=2, help="untimed calls before them")
    ap.add_argument("--seed", type=int, default=0, help="seed of the main code (n = 72, m = 72)")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip timing the CPU oracle")
    ap.add_argument("--cpu-seconds", type=float, default=30.0, help="time limit of the CPU oracle sample")
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
    ap.add_argument("--walk-only", action="store_true",
                    help="only run the plain per-round walk on the same code (--steps timed calls after "
                         "one warm-up call), for a profiler")
    ap.add_argument("--batch-only", action="store_true",
                    help="only run the config-4 batch leg (two batched calls and the per-code loop), for a profiler")
    ap.add_argument("--latency-only", action="store_true",
                    help="only run the time-to-exact-d leg on configs 1 and 2, for a profiler")
    ap.add_argument("--round-sweep", action="store_true",
                    help="only run one large round (48 two-row packages, t = 6) at D = 1..4 words per "
                         "half, for per-D kernel durations from a profiler")
    return ap.parse_args()


def cpu_baseline(G, field, budget_s):
    """The oracle's plain enumeration of the same code's rounds t = 1..6 on
    both generator matrices (about 2.9e9 codewords), stopped early once
    budget_s seconds have passed."""
    from oracle import oracle as O
    cores = min(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)), 16)
    B = O.expand(G, field)
    gs = O.gamma(B, O.DIAG_F4, 2, with_rows=True)
    done, visited, last = 0.0, 0, None
    for t in range(1, 7):
        for j, g in enumerate(gs):
            t0 = time.perf_counter()
            _, _, cnt = O.round_min(g["rows"], g["dims"], t, nthreads=cores)
            done += time.perf_counter() - t0
            visited += cnt
            last = (t, j + 1)
            if done >= budget_s:
                break
        if done >= budget_s:
            break
    return {"value": visited / done, "unit": "codewords/s", "cores": cores, "kind": "oracle",
            "sample": f"oracle enumeration of the same code, rounds t=1..{last[0]} on Gamma_1..Gamma_{last[1]}: "
                      f"{visited} codewords in {done:.2f} s wall on {cores} threads"}


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


def leg_batched(Q, W, a):
    codes, drawn = config4_codes(Q, W, a.batch_codes, a.batch_max_work)
    budget = int(a.batch_max_work * 4)
    import torch
    torch.cuda.synchronize()
    # The first call also fills the library's device-memory pool (tables of
    # every code); the timed call is the second, as the per-code loop below
    # runs with a warm pool too.
    t0 = time.perf_counter()
    Q.qd_distance_batch(codes, budget=budget)
    t_cold = time.perf_counter() - t0
    t0 = time.perf_counter()
    st, ds, wits, sts, stats = Q.qd_distance_batch(codes, budget=budget)
    t_batch = time.perf_counter() - t0
    comb_b = sum(s.combinations for s in stats)
    t0 = time.perf_counter()
    comb_p, ds_p = 0, []
    for G, f in codes:
        st1, d1, _, s1 = Q.qd_distance_ex(G, f, budget=budget)
        comb_p += s1.combinations
        ds_p.append(d1)
    t_plain = time.perf_counter() - t0
    ns = [G.shape[1] // 2 if f == 2 else G.shape[1] for G, f in codes]
    return {
        "workload": f"config 4: first {len(codes)} of {drawn} drawn codes (n~U{{24..96}}, even additive m~U{{n-8..n+8}}, "
                    f"odd F4-linear k=n/2) with planner-predicted work <= {a.batch_max_work:.0e}; budget {budget:.0e}",
        "codes": len(codes), "drawn": drawn, "n_range": [min(ns), max(ns)],
        "exact": sum(1 for x in sts if x == 0), "incomplete": sum(1 for x in sts if x == 1),
        "same_d_as_per_code": ds == ds_p,
        "batched_s": t_batch, "batched_codewords_per_s": comb_b / t_batch, "batched_first_call_s": t_cold,
        "per_code_s": t_plain, "per_code_codewords_per_s": comb_p / t_plain,
        "speedup": t_plain / t_batch,
    }


def leg_plain(Q, G, field, engine_step_ms, engine_combos):
    """The plain per-code GPU path on the same code: no saved sums, every
    lane unranks and XORs its whole combination."""
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
    walked = sum(s.words for s in runs) / runs[0].D  # codewords evaluated (one-row packages repeat)
    kernel_ms = sum(s.kernel_ms for s in runs)
    wall_ms = sum(s.wall_ms for s in runs)
    D = runs[0].D
    return {"d": d, "ms_per_step": wall_ms / steps, "codewords_per_s": combos / (wall_ms * 1e-3),
            "kernel_codewords_per_s": combos / (kernel_ms * 1e-3),
            "walked_per_combination": walked / combos,
            "launches_per_step": sum(s.launches for s in runs) / steps,
            # per walked codeword: 2D XOR + D OR + D v_bcnt + 1 min
            "roofline_frac_4D1_ops": walked * (4 * D + 1) / (kernel_ms * 1e-3) / PEAK_LANE_OPS,
            "engine_speedup": (wall_ms / steps) / engine_step_ms}


def leg_full_weight(Q, G, field, stream, steps):
    """The same code with every word of every codeword evaluated
    (partial_weight = -1): the enumeration rate without partial weights."""
    runs = []
    for i in range(steps + 1):
        st, d, wit, s = Q.qd_distance_ex(G, field, stream=stream, timing=1, partial_weight=-1)
        assert st == 0
        if i:
            runs.append(s)
    combos = sum(s.combinations for s in runs)
    enum = sum(s.enumerated for s in runs)
    words = sum(s.words for s in runs)
    kernel_ms = sum(s.kernel_ms for s in runs)
    enum_ms = sum(s.enumerated_kernel_ms for s in runs)
    wall_ms = sum(s.wall_ms for s in runs)
    return {"d": d, "ms_per_step": wall_ms / steps, "codewords_per_s": combos / (wall_ms * 1e-3),
            "kernel_codewords_per_s": combos / (kernel_ms * 1e-3),
            "roofline_frac": algorithmic_ops(words, enum) / (enum_ms * 1e-3) / PEAK_LANE_OPS}


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


def leg_serving(Q, W, a):
    """Config 5: Poisson arrivals, n log-uniform in 16..96, alternately
    additive (m = n) and F4-linear (k = n/2); requests whose predicted work
    exceeds 1e10 are redrawn (stated in the output)."""
    raw = W.config5(a.serve_requests * 4, 1.0)
    reqs, drawn = [], 0
    for _, G, f in raw:
        drawn += 1
        if predicted_work(Q, G, f) <= 1e10:
            reqs.append((G, f))
            if len(reqs) == a.serve_requests:
                break
    # service capacity: the same requests run back to back as one batch
    # (timed on a second call, after device memory and tables are warm)
    Q.qd_distance_batch(reqs)
    t0 = time.perf_counter()
    Q.qd_distance_batch(reqs)
    t_all = time.perf_counter() - t0
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
        Q.qd_engine_submit(e, G, f, i)
    while len(lat) < len(reqs):
        for r, w in Q.qd_engine_poll(e, 64, 100):
            lat.append(r.latency_ms); comb += r.combinations; statuses.append(r.status)
    t_total = time.perf_counter() - t_start
    Q.qd_engine_destroy(e)
    lat.sort()
    return {"workload": f"config 5: {len(reqs)} requests of {drawn} drawn (predicted work <= 1e10), "
                        f"Poisson rate {rate:.1f}/s (60% of back-to-back capacity)",
            "rate_per_s": rate, "requests": len(reqs), "exact": sum(1 for x in statuses if x == 0),
            "p50_ms": lat[len(lat) // 2], "p99_ms": lat[min(len(lat) - 1, int(0.99 * len(lat)))],
            "codewords_per_s": comb / t_total, "window_s": t_total}


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
    if a.batch_only:
        print(json.dumps({"batched": leg_batched(Q, W, a)}))
        return
    if a.latency_only:
        print(json.dumps({"latency": leg_latency(Q, W)}))
        return
    if a.walk_only:
        print(json.dumps({"walk_per_round": leg_walk(Q, G, field, stream.cuda_stream, float("nan"), a.steps)}))
        return

    def step():
        st, d, wit, s = Q.qd_distance_ex(G, field, stream=stream.cuda_stream, timing=1)
        if st != 0:
            raise RuntimeError(Q.qd_strerror(st))
        return d, s

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [step() for _ in range(a.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    d = stats[0][0]
    assert all(x[0] == d for x in stats)
    combos = sum(s.combinations for _, s in stats)
    kernel_ms = sum(s.kernel_ms for _, s in stats)
    launches = sum(s.launches for _, s in stats)
    D = stats[0][1].D
    # The roofline counts what the device enumerated (rounds run ahead
    # speculatively included) over the launch time spent on it.
    words = sum(s.words for _, s in stats)
    enum = sum(s.enumerated for _, s in stats)
    enum_ms = sum(s.enumerated_kernel_ms for _, s in stats)
    achieved = algorithmic_ops(words, enum) / (enum_ms * 1e-3)
    achieved_survey = (4 * words + enum) / (enum_ms * 1e-3)
    s0 = stats[0][1]
    out = {
        "metric": "codewords/s (XOR+symplectic wt) & time-to-exact-d",
        "value": combos / wall,
        "unit": "codewords/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": wall * 1e3 / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"single additive code n=72 m=72 Bernoulli(1/2), seed {a.seed} (config 3)",
                   "d": d, "diag": "F4" if s0.diag == 4 else "F2", "gammas": s0.h,
                   "packages": list(s0.P)[:s0.h], "delta": list(s0.delta)[:s0.h],
                   "rounds": s0.nlog, "codewords_per_step": combos // a.steps},
        "time_to_exact_d_ms": wall * 1e3 / a.steps,
        "host_ms_per_step": sum(s.host_ms for _, s in stats) / a.steps,
        "kernel_codewords_per_s": combos / (kernel_ms * 1e-3),
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_LANE_OPS / 1e12,
            "unit": "TOP/s",
            "frac": achieved / PEAK_LANE_OPS,
            "traffic": TRAFFIC["bytes_per_launch"] if kernel_fingerprint() == TRAFFIC["fingerprint"] else None,
            "kernel": f"qd_round_kernel<{D}>",
            "ops_per_codeword": algorithmic_ops(words, enum) / enum,
            "words_per_codeword": words / enum,
            "frac_4D1_ops": achieved_survey / PEAK_LANE_OPS,
            "launches": launches,
            "avg_launch_ms": enum_ms / max(launches, 1),
        },
        "device": name,
    }
    if a.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = src.numel() * 4
    if not a.no_extra:
        out["full_weight"] = leg_full_weight(Q, G, field, stream.cuda_stream, 5)
        out["plain_per_code"] = leg_plain(Q, G, field, wall * 1e3 / a.steps, combos / a.steps)
        out["walk_per_round"] = leg_walk(Q, G, field, stream.cuda_stream, wall * 1e3 / a.steps, 3)
        out["batched"] = leg_batched(Q, W, a)
        out["serving"] = leg_serving(Q, W, a)
        out["latency"] = leg_latency(Q, W)
        out["constructions"] = leg_constructions(Q, W)
        out["stabilizer"] = leg_stabilizer(Q, W, a)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(G, field, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
