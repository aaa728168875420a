"""Benchmark: Kawasaki swap attempts per second on a 4096x4096 bit-packed lattice.

One step is one pass of the hot path over the standing 4096^2 workload
(composition 0.5, omega = 0.88 kT, bit-packed, lattice resident in HBM):
10,000 sweeps (N = 16.8 M attempts each), then N_AB and the cluster-size
histogram of species 1.  The line also carries:
  * roofline -- the sweep kernel's algorithmic integer-op rate against the
    VALU peak, and its algorithmic bytes against HBM peak (measured with HIP
    events around every sweep launch on the library's stream);
  * cpu_baseline -- the CPU oracle timed on a bounded sample of the same
    workload on this host;
  * batched -- aggregate attempts/s of the batch engine against the same
    replicas run one after another through the plain path; batched_offgrid
    -- the same with the int8 replicas' sides rounded to multiples of 4;
  * grid_400 -- the 12-run 400x400 grid batched, histograms every 1000 sweeps;
  * serving -- p50/p99 latency, served and offered attempts/s of the job
    server replaying the Poisson job trace, saturated and below saturation;
  * triangular -- the paper's own six-neighbour helical lattice (4092^2,
    int8): attempts/s, the tile kernel's time per launch and its roofline,
    with the triangular CPU oracle timed beside it; and 256 replicas of the
    paper's 100 x 100 lattice batched against one after another;
  * mpkk -- the paper's literal MPKK (7-site domain cover, synchronous
    iterations) on a 4098 x 4095 ring: attempts/s, roofline, oracle; and its
    bias: the equilibrium unlike-bond fraction against the exact conflict-free
    chain on a 1020 x 1036 ring, omega 0.1 .. 0.5.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks and unit counts
HBM_PEAK_GBS = 8000.0
CUS, LANES, CLOCK_HZ = 256, 64, 2.4e9
# VALU peak: 256 CUs x 4 SIMDs x 16 lanes per clock = one fp32 FMA per lane per
# clock (the published 157.3 TFLOP/s counts an FMA as two flops and uses the
# packed two-wide form).  It is the roofline's unit: every algorithmic
# instruction is priced at its measured issue cost relative to an fp32 FMA.
VALU_PEAK_GOPS = CUS * LANES * CLOCK_HZ / 1e9   # fp32-FMA-equivalent lane-ops/s

# Algorithmic instruction mix of one attempt, in 32-bit VALU lane-ops by kind
# (one lane-op = one instruction on one lane).  "fast" is the bitwise/add
# class (v_xor, v_and, v_or, v_bitop3, v_add, v_xnor), which gfx950 issues in
# about 0.6 of the cycles of an FMA; v_mad_u64_u32, v_alignbit, v_mul and
# v_bcnt issue at the FMA rate (kk_valu_issue_cycles measures both on the box).
# Square torus, bit-sliced sweep:
#   random planes: 3 Philox4x32-10 blocks per 32-site word per sweep, 10 rounds
#     x (2 v_mad_u64_u32 + 2 three-input xors)         -> 60 mad + 60 fast / 32
#   acceptance planes: 3 bit-sliced 10-bit compares per word per sweep, 25 ops
#     each (a borrow op and an XNOR per bit, a 5-op AND tree)   -> 75 fast / 32
#   decision of the 8 centres of a word in one phase: 9 funnel shifts (8
#     neighbour alignments, the class mask), 28 selects/counter/threshold ops;
#     applying the accepted exchanges: 4 direction splits, 2 shifts, 1 xor3, 2
#     edge tests; counting: 1 and, 1 popcount, 1 add          -> per word-phase
#     9 alignbit + 37 fast + 2 shift + 1 bcnt, over 8 attempts
SQUARE_MIX = {"mad_u64_u32": 60 / 32, "alignbit": 9 / 8, "lshl": 2 / 8, "bcnt": 1 / 8,
              "fast": (60 + 75) / 32 + 37 / 8}
OPS_PER_ATTEMPT = sum(SQUARE_MIX.values())


def valu_weights(cycles):
    """Issue cost of each instruction kind relative to an fp32 FMA, from the
    measured cycles per wave64 instruction (None: every kind at the FMA rate)."""
    if not cycles:
        return {k: 1.0 for k in ("mad_u64_u32", "alignbit", "lshl", "bcnt", "mul_lo", "fast")}
    f = cycles["fma_f32"]
    fast = (cycles["xor"] + cycles["bitop3"] + cycles["add"]) / 3.0
    return {"mad_u64_u32": cycles["mad_u64_u32"] / f, "alignbit": cycles["alignbit"] / f,
            "lshl": cycles["lshl"] / f, "bcnt": cycles["bcnt"] / f, "mul_lo": cycles["mul_lo"] / f,
            "fast": fast / f}


def weighted_ops(mix, weights):
    return sum(n * weights[k] for k, n in mix.items())


def roofline_alu(mix, weights, attempts_per_s):
    """The roofline entry of a VALU-bound kernel at the given attempt rate."""
    w = weighted_ops(mix, weights)
    ops = w * attempts_per_s / 1e9
    return {"bound": "alu", "achieved": round(ops / 1e3, 3), "peak": round(VALU_PEAK_GOPS / 1e3, 3),
            "unit": "TOP/s (fp32-FMA-equivalent VALU lane-ops)", "frac": round(ops / VALU_PEAK_GOPS, 4),
            "ops_per_attempt": round(sum(mix.values()), 3), "weighted_ops_per_attempt": round(w, 3),
            "instruction_mix": {k: round(v, 4) for k, v in mix.items()}}


# HBM-side bytes per launch of the sweep kernel on this workload, from the
# rocprofv3 FETCH_SIZE / WRITE_SIZE passes recorded in
# profiles/halo_kernel_4096_bitpacked.md (counters scaled by what they read for
# a plain copy kernel of known size).  Valid only for the kernel sources that
# were profiled: the line reports null once they change.
PROFILED_TRAFFIC = {"sources_sha256_prefix": "b3cfdf93ff201d3a", "tile": (16, 128, 2),
                    "bytes_per_launch": 4721976}
KERNEL_SOURCES = ["kk_sweep.hip", "kk_common.hpp", "kk_kernels.hpp"]
# The same for the triangular whole-sweep tile kernel on the 4092^2 lattice with
# 256 x 256 tiles (profiles/tri_tile_sweep_4092.md).
TRI_PROFILED_TRAFFIC = {"sources_sha256_prefix": "acfed7f9645a8c30", "tile": (256, 256),
                        "bytes_per_launch": 35863064}
TRI_KERNEL_SOURCES = ["kk_tri.hip", "kk_tri.hpp", "kk_common.hpp"]
# And for the literal-MPKK whole-step tile kernel on the 4098 x 4095 ring with
# 257 x 256 tiles (profiles/mpkk_tile_step_4098x4095.md).
MPKK_PROFILED_TRAFFIC = {"sources_sha256_prefix": "acfed7f9645a8c30", "tile": (257, 256),
                         "bytes_per_launch": 35132607}
# The 400^2 int8 paths (profiles/halo_kernel_400_int8.md): the plain sweep
# kernel with 2 x 16 tiles, and the batch tile kernel at the autotuner's 16 x 28
# tiles, one unit per thread, over the 12 runs.
GRID_PROFILED_TRAFFIC = {"sources_sha256_prefix": "b3cfdf93ff201d3a", "plain_tile": (2, 16, 1),
                         "plain_bytes_per_launch": 886838, "batch_tile": (16, 28),
                         "batch_bytes_per_launch": 6599810}


def kernel_sources_sha(files=KERNEL_SOURCES) -> str:
    import hashlib

    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1309_4349_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


BYTES_PER_ATTEMPT_BITS = 0.25   # read + write one bit per site per sweep
BYTES_PER_ATTEMPT_INT8 = 2.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(job, budget_s: float = 12.0):
    """Time the CPU oracle (as it stands) on whole sweeps of the same lattice."""
    import numpy as np

    import oracle

    threads = oracle.set_threads(0)
    s = oracle.init(job.L, job.composition, job.seed)
    t0 = time.perf_counter()
    oracle.sweeps(s, job.omega, job.seed, 0, 1)
    one = time.perf_counter() - t0
    n = max(1, int(budget_s / max(one, 1e-3)) - 1)
    t0 = time.perf_counter()
    oracle.sweeps(s, job.omega, job.seed, 1, n)
    dt = time.perf_counter() - t0
    rate = n * job.L * job.L / dt
    # the same on one core, over about a third of the budget
    oracle.set_threads(1)
    t0 = time.perf_counter()
    oracle.sweeps(s, job.omega, job.seed, 1 + n, 1)
    one1 = time.perf_counter() - t0
    n1 = max(1, int(budget_s / 3 / max(one1, 1e-3)))
    t0 = time.perf_counter()
    oracle.sweeps(s, job.omega, job.seed, 2 + n, n1)
    dt1 = time.perf_counter() - t0
    oracle.set_threads(threads)
    return {"value": rate, "unit": "attempts/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} sweeps of the {job.L}x{job.L} x={job.composition} omega={job.omega} lattice "
                      f"({n * job.L * job.L:.3e} attempts, {dt:.1f} s, sweeps 1..{n})",
            "single_core": {"value": n1 * job.L * job.L / dt1, "cores": 1,
                            "sample": f"{n1} further sweeps ({dt1:.1f} s)"}}


def classical_baseline(budget_s: float = 4.0):
    """The paper's "classical computation": sequential random-site Kawasaki
    (a random site, a random one of its 4 neighbours, Metropolis on the energy
    recount) on one core, timed on the 4096^2 and one 400^2 workload."""
    import oracle
    from paper_1309_4349_amd import workloads as wl

    out = {"kind": "oracle (sequential random-site Kawasaki)", "cores": 1, "unit": "attempts/s"}
    for key, job in (("L4096", wl.big_4096()), ("L400", wl.grid_400()[5])):
        s = oracle.init(job.L, job.composition, job.seed)
        n = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s:
            oracle.seq_kawasaki(s, job.omega, job.seed + n, 1)
            n += 1
        dt = time.perf_counter() - t0
        out[key] = {"value": n * job.L * job.L / dt,
                    "sample": f"{n} sweeps ({n * job.L * job.L:.3e} attempts, {dt:.1f} s) of {job.tag}"}
        log(f"[bench] classical sequential Kawasaki {job.L}^2: {out[key]['value']:.3e} attempts/s on one core")
    out["paper_context"] = ("the paper reports its GPU code (Tesla M2090, CUDA 4.1) up to about 55x faster than "
                            "its sequential CPU computation (Xeon E5640, 2.67 GHz); different hardware, lattice "
                            "and algorithm: context only")
    return out


def small_64(cpu: bool):
    """The 64x64 workload (x = 0.5, omega = 0.5, 1000 sweeps, then N_AB and
    the species-1 histogram): GPU seconds, and the oracle's CPU seconds on one
    core for the same run."""
    import torch

    from paper_1309_4349_amd import kk
    from paper_1309_4349_amd import workloads as wl

    job = wl.small_64()
    sim = kk.Sim(job.L, job.composition, job.omega, job.seed, layout=job.layout)
    sim.sweep(2)
    sim.restart()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.sweep(job.sweeps)
    sim.energy()
    sim.cluster_hist(1)
    torch.cuda.synchronize()
    gpu_s = time.perf_counter() - t0
    sim.close()
    out = {"workload": job.tag + ", then N_AB and the species-1 histogram", "gpu_s": gpu_s,
           "gpu_attempts_per_s": job.attempts / gpu_s}
    if cpu:
        import oracle

        threads = oracle.set_threads(0)  # the current count, restored below
        oracle.set_threads(1)
        s = oracle.init(job.L, job.composition, job.seed)
        t0 = time.perf_counter()
        oracle.sweeps(s, job.omega, job.seed, 0, job.sweeps)
        oracle.energy(s)
        oracle.cluster_hist(s, 1)
        out["oracle_cpu_s"] = time.perf_counter() - t0
        out["oracle_cores"] = 1
        oracle.set_threads(threads)
    log(f"[bench] 64^2 config: GPU {gpu_s * 1e3:.2f} ms, oracle {out.get('oracle_cpu_s', float('nan')):.2f} s")
    return out


# Algorithmic mix of one attempt on the triangular lattice: one Philox4x32-10
# block per two sites (10 mad + 10 fast: a block's words 0-1 serve the even
# site of a pair and words 2-3 the odd one, so a kernel that computes a whole
# block per centre does twice the method's random-number work), the partner
# direction (one multiply-high) and uniform (2 fast), 12 neighbour addresses
# (24), 12 unlike tests and their sum (24), the threshold lookup and compare
# (3), the swap (2) -> 76.  Algorithmic bytes: each site read and written once
# per sweep (2 B).  The whole-sweep tile kernel recomputes a halo on top of this.
TRI_MIX = {"mad_u64_u32": 10.0, "mul_lo": 1.0, "fast": 65.0}
TRI_OPS_PER_ATTEMPT = sum(TRI_MIX.values())


def tri_batch(n: int, L: int, sweeps: int, n_plain: int):
    """Many replicas of the paper's 100 x 100 triangular lattice in one batch
    (each ring held whole in one workgroup), against the same replicas run one
    after another through the single-lattice path."""
    from dataclasses import dataclass

    import torch

    from paper_1309_4349_amd import kk

    @dataclass
    class Rep:
        L: int
        composition: float
        omega: float
        seed: int
        sweeps: int

    jobs = [Rep(L, 0.2 + 0.6 * (i % 7) / 6, 0.2 + 1.2 * (i % 13) / 12, 0x13094349 + i, sweeps) for i in range(n)]
    b = kk.TriBatch(jobs)
    info = b.info()
    b.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    b.close()
    rate = n * L * L * sweeps / dt
    sims = [kk.Sim(j.L, j.composition, j.omega, j.seed, geometry="triangular") for j in jobs[:n_plain]]
    for s_ in sims:
        s_.sweep(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s_ in sims:
        s_.sweep(sweeps)
    torch.cuda.synchronize()
    dtp = time.perf_counter() - t0
    for s_ in sims:
        s_.close()
    plain = n_plain * L * L * sweeps / dtp
    log(f"[bench] triangular batch {n} x {L}^2: {rate:.3e} attempts/s, one after another {plain:.3e} "
        f"({rate / plain:.1f}x) {info}")
    return {"workload": f"{n} triangular {L}x{L} replicas, x in [0.2, 0.8], omega in [0.2, 1.4], {sweeps} sweeps each",
            "batched_attempts_per_s": rate, "plain_attempts_per_s": plain, "plain_replicas_timed": n_plain,
            "speedup": rate / plain, "layout": info}


def triangular(sweeps: int, profile_sweeps: int, cpu: bool, batch_sweeps: int = 1000, weights=None):
    """Attempts/s of the triangular helical lattice (the paper's geometry)."""
    import torch

    import oracle
    from paper_1309_4349_amd import kk

    L, x, w, seed = 4092, 0.5, 0.88, 0x13094349
    N = L * L
    sim = kk.Sim(L, x, w, seed, geometry="triangular")
    sim.sweep(5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.sweep(sweeps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rate = sweeps * N / dt
    sim_tile = sim.tri_get_tile()
    ms, launches = sim.sweep_timed(profile_sweeps)
    per_launch_s = ms / 1e3 / launches
    per_launch = N * profile_sweeps / launches
    hbm = BYTES_PER_ATTEMPT_INT8 * per_launch / per_launch_s / 1e9
    nab, _ = sim.energy()
    sim.close()
    traffic = None
    if (kernel_sources_sha(TRI_KERNEL_SOURCES) == TRI_PROFILED_TRAFFIC["sources_sha256_prefix"]
            and tuple(sim_tile) == TRI_PROFILED_TRAFFIC["tile"]):
        traffic = TRI_PROFILED_TRAFFIC["bytes_per_launch"]
    out = {"workload": f"triangular helical {L}x{L} int8, x={x}, omega={w}, {sweeps} sweeps",
           "value": rate, "unit": "attempts/s", "n_unlike_over_3N": nab / (3 * N),
           "roofline": {**roofline_alu(TRI_MIX, weights, per_launch / per_launch_s),
                        "traffic": traffic, "kernel": "tri_tile_sweep" if sim_tile[0] else "tri_phase",
                        "kernel_us": round(per_launch_s * 1e6, 3), "launches": int(launches),
                        "tile": {"cols": sim_tile[0], "rows": sim_tile[1]},
                        "hbm_achieved_GBps": round(hbm, 1), "hbm_frac": round(hbm / HBM_PEAK_GBS, 5)}}
    log(f"[bench] triangular {L}^2: {rate:.3e} attempts/s, {per_launch_s * 1e6:.2f} us/launch")
    out["batch"] = tri_batch(256, 100, batch_sweeps, 32)
    if cpu:
        threads = oracle.set_threads(0)
        s = oracle.init(L, x, seed)
        t0 = time.perf_counter()
        oracle.tri_sweeps(s, w, seed, 0, 1)
        one = time.perf_counter() - t0
        n = max(1, int(8.0 / max(one, 1e-3)) - 1)
        t0 = time.perf_counter()
        oracle.tri_sweeps(s, w, seed, 1, n)
        dtc = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": n * N / dtc, "unit": "attempts/s", "cores": threads, "kind": "oracle",
                               "sample": f"{n} sweeps of the same {L}x{L} triangular lattice ({dtc:.1f} s)"}
        log(f"[bench] triangular oracle {n * N / dtc:.3e} attempts/s on {threads} threads")
    return out


# One literal-MPKK attempt: one Philox block per two domains (10 mad + 10
# fast), k draw amortised (0), direction (one multiply-high) and uniform (2),
# 12 neighbour indices (24), 12 unlike tests and their sum (24), threshold (3),
# writing the domain's result (13) -> 87.
MPKK_MIX = {"mad_u64_u32": 10.0, "mul_lo": 1.0, "fast": 76.0}
MPKK_OPS_PER_ATTEMPT = sum(MPKK_MIX.values())


def mpkk(steps: int, bias_steps: int, cpu: bool, weights=None):
    """Throughput of the literal MPKK and its bias against the exact chain."""
    import math

    import numpy as np
    import torch

    import oracle
    from paper_1309_4349_amd import kk

    L, H, x, w, seed = 4098, 4095, 0.5, 0.88, 0x13094349
    N = L * H
    sim = kk.Sim(L, x, w, seed, geometry="triangular", rows=H, scheme="mpkk")
    sim.sweep(3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.sweep(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rate = steps * N / dt
    mp_tile = sim.tri_get_tile()
    ms, launches = sim.sweep_timed(50)
    per_launch_s = ms / 1e3 / launches
    per_launch = N * 50 / launches
    hbm = BYTES_PER_ATTEMPT_INT8 * per_launch / per_launch_s / 1e9
    sim.close()
    traffic = None
    if (kernel_sources_sha(TRI_KERNEL_SOURCES) == MPKK_PROFILED_TRAFFIC["sources_sha256_prefix"]
            and tuple(mp_tile) == MPKK_PROFILED_TRAFFIC["tile"]):
        traffic = MPKK_PROFILED_TRAFFIC["bytes_per_launch"]
    out = {"workload": f"literal MPKK, triangular helical {L}x{H} int8, x={x}, omega={w}, {steps} steps",
           "value": rate, "unit": "attempts/s",
           "roofline": {**roofline_alu(MPKK_MIX, weights, per_launch / per_launch_s),
                        "traffic": traffic, "kernel": "mpkk_tile_step" if mp_tile[0] else "mpkk_iter",
                        "kernel_us": round(per_launch_s * 1e6, 3), "launches": int(launches),
                        "tile": {"cols": mp_tile[0], "rows": mp_tile[1]},
                        "hbm_achieved_GBps": round(hbm, 1), "hbm_frac": round(hbm / HBM_PEAK_GBS, 5)}}
    log(f"[bench] mpkk {L}x{H}: {rate:.3e} attempts/s, {per_launch_s * 1e6:.2f} us/launch")
    if cpu:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        s = oracle.init_rect(L, H, x, seed)
        t0 = time.perf_counter()
        n = 0
        while time.perf_counter() - t0 < 6.0:
            oracle.mpkk_steps(s, w, seed, n, 1)
            n += 1
        dtc = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": n * N / dtc, "unit": "attempts/s", "cores": 1, "kind": "oracle",
                               "sample": f"{n} steps of the same {L}x{H} ring ({dtc:.1f} s, single-threaded)"}
        log(f"[bench] mpkk oracle {n * N / dtc:.3e} attempts/s")
    if bias_steps <= 0:
        return out
    # bias: equilibrium N_AB / 3N on a 1020 x 1036 ring (both schedules are defined on it), both
    # schemes from the same random start; the drift between the two halves of the measured
    # stretch shows whether the run was in equilibrium
    bias = []
    L, H = 1020, 1036
    N = L * H
    for omega in (0.1, 0.2, 0.3, 0.4, 0.5):
        row = {"omega": omega}
        for scheme in ("classes", "mpkk"):
            sim = kk.Sim(L, 0.5, omega, 11, geometry="triangular", rows=H, scheme=scheme)
            sim.sweep(3000)
            v = []
            for _ in range(bias_steps // 30):
                sim.sweep(30)
                v.append(sim.energy()[0] / (3 * N))
            sim.close()
            v = np.array(v[: len(v) // 20 * 20])
            bm = v.reshape(20, -1).mean(1)
            half = len(v) // 2
            row[scheme] = {"f_unlike": float(bm.mean()), "stderr": float(bm.std(ddof=1) / math.sqrt(20)),
                           "drift": float(v[half:].mean() - v[:half].mean())}
        row["mpkk_minus_exact"] = row["mpkk"]["f_unlike"] - row["classes"]["f_unlike"]
        row["sigma"] = row["mpkk_minus_exact"] / math.hypot(row["mpkk"]["stderr"], row["classes"]["stderr"])
        log(f"[bench] mpkk bias at omega={omega}: {row['mpkk_minus_exact']:+.5f} ({row['sigma']:.1f} sigma), "
            f"drift {row['classes']['drift']:+.5f} / {row['mpkk']['drift']:+.5f}")
        bias.append(row)
    out["bias"] = {"workload": f"{L}x{H} ring, x=0.5, 3000 burn-in + {bias_steps} measured steps each, "
                               "20 batch means; drift = second-half minus first-half mean", "rows": bias}
    return out


def batched_vs_plain(sweeps: int, plain_sweeps: int, offgrid: bool = False):
    """Aggregate attempts/s of the 256-replica table: one batch run against the
    same replicas advanced one after another through the plain path.  With
    `offgrid`, the int8 replicas keep sides that are multiples of 4 (most are
    not whole 32-site words), so they run on the batch's tile kernel rather
    than its whole-lattice resident kernels."""
    import torch

    from paper_1309_4349_amd import kk
    from paper_1309_4349_amd import workloads as wl

    jobs = wl.batch_replicas(n=256, sweeps=sweeps, offgrid=offgrid)
    sites = sum(j.L * j.L for j in jobs)
    b = kk.Batch(jobs)
    info = b.info()
    tw, th, tms = b.autotune(10)
    info["tile_words"], info["tile_rows"] = tw, th
    log(f"[bench] batch autotune: tiles of at most {tw} words x {th} rows ({tms:.3f} ms per sweep)")
    b.run()   # warm-up run
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run()
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    batched_rate = sites * sweeps / tb
    log(f"[bench] batch: {len(jobs)} replicas x {sweeps} sweeps in {tb:.3f} s = {batched_rate:.3e} attempts/s {info}")
    b.close()
    sims = [kk.Sim(j.L, j.composition, j.omega, j.seed, layout=j.layout) for j in jobs]
    for s in sims:
        s.sweep(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in sims:
        s.sweep(plain_sweeps)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    plain_rate = sites * plain_sweeps / tp
    log(f"[bench] plain: {len(jobs)} replicas one at a time x {plain_sweeps} sweeps in {tp:.3f} s = "
        f"{plain_rate:.3e} attempts/s")
    for s in sims:
        s.close()
    rounding = ("int8 replicas multiples of 4, bit-packed multiples of 32" if offgrid else "multiples of 32")
    return {"workload": f"256 replicas, L log-uniform 64..1024 ({rounding}), x~U[0.2,0.8], omega~U[0.2,1.4]",
            "sites": sites, "batched_sweeps": sweeps, "batched_attempts_per_s": batched_rate,
            "batched_s": tb, "plain_sweeps_per_replica": plain_sweeps, "plain_attempts_per_s": plain_rate,
            "plain_s": tp, "speedup": batched_rate / plain_rate, "plan": info}


def grid_400(rounds: int, every: int, weights=None, tile=None):
    """The 12-run 400x400 grid (3 compositions x 4 omegas, int8) advanced together
    in one batch, with every run's species-1 cluster histogram taken every
    `every` sweeps, against the same runs advanced one after another; and the
    rooflines of the plain single-lattice sweep kernel and of the batch.
    `tile` (words, rows, units per thread) fixes the batch tile instead of
    autotuning it, so that profiler runs all time the same tile."""
    import torch

    from paper_1309_4349_amd import kk
    from paper_1309_4349_amd import workloads as wl

    jobs = wl.grid_400(sweeps=every)
    sites = sum(j.L * j.L for j in jobs)
    b = kk.Batch(jobs)
    if tile:
        b.set_tile(*tile)
        tw, th = tile[0], tile[1]
    else:
        tw, th, _ = b.autotune(20)
    plan = b.info()
    # warm-up rounds: in a process that has loaded torch, the first few
    # labelling rounds after the batch is built take several ms longer
    for _ in range(4):
        b.run()
        b.cluster_hists(1)
        for i in range(len(jobs)):
            b.sim(i).cluster_hist(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(rounds):
        b.run()
        b.cluster_hists(1)  # every run's labelling, one device wait
        for i in range(len(jobs)):
            b.sim(i).cluster_hist(1)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    # the sweeps alone (no histograms), for the batch's roofline
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run()
    torch.cuda.synchronize()
    tsw = time.perf_counter() - t0
    b.close()
    rate = sites * every * rounds / tb
    sims = [kk.Sim(j.L, j.composition, j.omega, j.seed, layout=j.layout) for j in jobs]
    for s in sims:
        s.sweep(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in sims:
        s.sweep(every)
        s.cluster_hist(1)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    # the plain path's sweep kernel on one 400^2 lattice, timed on the library's stream
    ms, launches = sims[5].sweep_timed(500)
    per_launch_s = ms / 1e3 / launches
    ptile = sims[5].get_tile()
    for s in sims:
        s.close()
    plain = sites * every / tp
    n1 = jobs[0].L * jobs[0].L
    same_src = kernel_sources_sha() == GRID_PROFILED_TRAFFIC["sources_sha256_prefix"]
    plain_roof = {**roofline_alu(SQUARE_MIX, weights, n1 / per_launch_s),
                  "traffic": GRID_PROFILED_TRAFFIC["plain_bytes_per_launch"]
                  if same_src and tuple(ptile) == GRID_PROFILED_TRAFFIC["plain_tile"] else None,
                  "kernel": f"halo_kernel<int8, {ptile[0]}, {ptile[2]}>", "kernel_us": round(per_launch_s * 1e6, 3),
                  "launches": int(launches), "tile": {"words": ptile[0], "rows": ptile[1], "units_per_thread": ptile[2]},
                  "algorithmic_bytes_per_launch": int(BYTES_PER_ATTEMPT_INT8 * n1),
                  "hbm_achieved_GBps": round(BYTES_PER_ATTEMPT_INT8 * n1 / per_launch_s / 1e9, 1),
                  "hbm_frac": round(BYTES_PER_ATTEMPT_INT8 * n1 / per_launch_s / 1e9 / HBM_PEAK_GBS, 5)}
    batch_sweep_rate = sites * every / tsw
    batch_roof = {**roofline_alu(SQUARE_MIX, weights, batch_sweep_rate),
                  "traffic": GRID_PROFILED_TRAFFIC["batch_bytes_per_launch"]
                  if same_src and (tw, th) == GRID_PROFILED_TRAFFIC["batch_tile"] else None,
                  "algorithmic_bytes_per_launch": int(BYTES_PER_ATTEMPT_INT8 * sites),
                  "kernel": "batch_tile_kernel (whole batch run of the 12 lattices, launch gaps included)",
                  "us_per_sweep": round(tsw / every * 1e6, 3), "plan": plan}
    log(f"[bench] 400^2 grid: batched {rate:.3e} attempts/s (tiles <= {tw}x{th}; sweeps alone "
        f"{batch_sweep_rate:.3e}, {tsw / every * 1e6:.1f} us per sweep of all 12), one after another {plain:.3e}; "
        f"plain sweep kernel {per_launch_s * 1e6:.2f} us per 400^2 sweep")
    return {"workload": "12 runs of 400x400 int8, x in {0.3,0.5,0.7} x omega in {0.3,0.6,0.9,1.2}, "
                        f"histogram of every run every {every} sweeps",
            "batched_attempts_per_s": rate, "rounds": rounds, "sweeps_per_round": every,
            "tile_words": tw, "tile_rows": th, "sequential_attempts_per_s": plain, "speedup": rate / plain,
            "batched_sweeps_only_attempts_per_s": batch_sweep_rate, "roofline_batched": batch_roof,
            "roofline_plain_single": plain_roof}


def serving(n_saturated: int, n_light: int, light_rate: float, chunk: int):
    """Replay the Poisson job trace through the job server: once at its own
    arrival rate (200 jobs/s, far above what one GPU serves) and once at a rate
    below saturation."""
    from paper_1309_4349_amd import serve
    from paper_1309_4349_amd import workloads as wl

    out = {"workload": "Poisson arrivals, L uniform over {128,256,512,1024,2048}, sweeps log-uniform 1e3..1e5, "
                       "x~U[0.2,0.8], omega~U[0.2,1.4]", "chunk_sweeps": chunk}
    sat = wl.serving_trace(n_jobs=n_saturated, rate=200.0)
    log(f"[bench] serving: {len(sat)} jobs at 200 jobs/s")
    out["saturated"] = serve.run_trace(sat, chunk_sweeps=chunk, log=None)
    log(f"[bench] serving saturated: {out['saturated']}")
    if n_light:
        light = wl.serving_trace(n_jobs=n_light, rate=light_rate, seed=wl.MASTER_SEED ^ 5)
        log(f"[bench] serving: {len(light)} jobs at {light_rate} jobs/s")
        out["below_saturation"] = serve.run_trace(light, chunk_sweeps=chunk, log=None)
        log(f"[bench] serving below saturation: {out['below_saturation']}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sweeps", type=int, default=10_000, help="sweeps per step")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-plain comparison")
    ap.add_argument("--batch-sweeps", type=int, default=10_000, help="sweeps per replica in the batch run")
    ap.add_argument("--batch-plain-sweeps", type=int, default=500,
                    help="sweeps per replica for the one-at-a-time plain baseline")
    ap.add_argument("--grid-rounds", type=int, default=10, help="rounds of 1000 sweeps for the 400^2 grid")
    ap.add_argument("--no-serve", action="store_true", help="skip the job-server trace replay")
    ap.add_argument("--serve-jobs", type=int, default=200, help="jobs of the saturated serving trace")
    ap.add_argument("--serve-light-jobs", type=int, default=60, help="jobs of the below-saturation trace")
    ap.add_argument("--serve-light-rate", type=float, default=5.0, help="arrival rate of the below-saturation trace")
    ap.add_argument("--serve-chunk", type=int, default=1000, help="sweeps per server step")
    ap.add_argument("--profile-sweeps", type=int, default=500, help="sweeps timed per launch for the roofline")
    ap.add_argument("--no-tri", action="store_true", help="skip the triangular-lattice measurement")
    ap.add_argument("--tri-sweeps", type=int, default=500, help="sweeps of the 4092^2 triangular lattice")
    ap.add_argument("--tri-batch-sweeps", type=int, default=1000, help="sweeps of each 100^2 replica in the batch")
    ap.add_argument("--no-mpkk", action="store_true", help="skip the literal-MPKK measurement")
    ap.add_argument("--mpkk-steps", type=int, default=500, help="MPKK steps of the 4098 x 4095 ring")
    ap.add_argument("--mpkk-bias-steps", type=int, default=6000, help="measured steps per bias run (0 skips the bias runs)")
    ap.add_argument("--grid-tile", default="",
                    help="words,rows,units_per_thread: fix the 400^2 batch tile instead of autotuning it")
    ap.add_argument("--grid-only", action="store_true",
                    help="only the 400^2 grid measurement (its JSON on one line), for profiling that path")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this size (counter calibration) and exit")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (independent replicas "
              "would be spread over GPUs, one process each; one large lattice would be split into row "
              "strips with a halo exchange per sweep)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1309_4349_amd import kk
    from paper_1309_4349_amd import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)            # device-to-device copy (runtime copy kernel)
        for _ in range(3):
            torch.neg(a, out=b)   # elementwise kernel: reads and writes n * 4 bytes
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 4}))
        return

    # issue cost of each instruction kind on this device (prices the rooflines)
    try:
        cycles = kk.valu_issue_cycles()
    except kk.KKError as e:
        log(f"[bench] VALU probe failed ({e}): every instruction priced at the FMA rate")
        cycles = None
    weights = valu_weights(cycles)
    log(f"[bench] VALU issue cycles per wave64 instruction: {cycles}")

    if args.grid_only:
        tile = tuple(int(v) for v in args.grid_tile.split(",")) if args.grid_tile else None
        print(json.dumps({"grid_400": grid_400(args.grid_rounds, 1000, weights, tile)}), flush=True)
        return

    job = wl.big_4096(args.sweeps)
    N = job.L * job.L
    log(f"[bench] creating {job.tag}")
    sim = kk.Sim(job.L, job.composition, job.omega, job.seed, layout="bitpacked")

    def step():
        sim.sweep(job.sweeps)
        sim.energy()
        sim.cluster_hist(1)

    for i in range(args.warmup):
        step()
        log(f"[bench] warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        log(f"[bench] step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    attempts = args.steps * job.sweeps * N
    value = attempts / dt
    nab, _ = sim.energy()
    log(f"[bench] {value:.4e} attempts/s, N_AB/2N = {nab / (2 * N):.5f}")

    # roofline of the sweep kernel: HIP events around every launch on the library's stream
    ms, launches = sim.sweep_timed(args.profile_sweeps)
    per_launch_s = ms / 1e3 / launches
    attempts_per_launch = N * args.profile_sweeps / launches
    hbm = BYTES_PER_ATTEMPT_BITS * attempts_per_launch / per_launch_s / 1e9
    tw, th, ku = sim.get_tile()
    traffic = None
    if (kernel_sources_sha() == PROFILED_TRAFFIC["sources_sha256_prefix"]
            and (tw, th, ku) == PROFILED_TRAFFIC["tile"] and job.L == 4096):
        traffic = PROFILED_TRAFFIC["bytes_per_launch"]
    roofline = {**roofline_alu(SQUARE_MIX, weights, attempts_per_launch / per_launch_s), "traffic": traffic,
                "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "algorithmic_bytes_per_launch": int(BYTES_PER_ATTEMPT_BITS * attempts_per_launch),
                "kernel": f"halo_kernel<bitpacked, {tw}, {ku}>",
                "kernel_us": round(per_launch_s * 1e6, 3), "launches": int(launches),
                "hbm_achieved_GBps": round(hbm, 1), "hbm_peak_GBps": HBM_PEAK_GBS,
                "hbm_frac": round(hbm / HBM_PEAK_GBS, 5),
                "tile": {"words": tw, "rows": th, "units_per_thread": ku},
                "valu_issue_cycles": {k: round(v, 3) for k, v in (cycles or {}).items()},
                "weights_rel_fma": {k: round(v, 3) for k, v in weights.items()}}
    log(f"[bench] sweep kernel {per_launch_s * 1e6:.2f} us/launch, frac {roofline['frac']}, "
        f"{hbm:.1f} GB/s algorithmic")
    # observables of the final state (labelling, N_AB and the random-neighbour draw)
    sim.sweep(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    obs = sim.observe(1)
    observe_ms = (time.perf_counter() - t0) * 1e3
    log(f"[bench] observables in {observe_ms:.2f} ms: {obs}")
    sim.close()

    batched = batched_off = None
    if not args.no_batch:
        batched = batched_vs_plain(args.batch_sweeps, args.batch_plain_sweeps)
        batched_off = batched_vs_plain(args.batch_sweeps, args.batch_plain_sweeps, offgrid=True)

    grid = None
    if not args.no_batch:
        grid = grid_400(args.grid_rounds, 1000, weights)

    served = None
    if not args.no_serve:
        served = serving(args.serve_jobs, args.serve_light_jobs, args.serve_light_rate, args.serve_chunk)

    tri = None
    if not args.no_tri:
        tri = triangular(args.tri_sweeps, 100, not args.no_cpu, args.tri_batch_sweeps, weights)

    mp = None
    if not args.no_mpkk:
        mp = mpkk(args.mpkk_steps, args.mpkk_bias_steps, not args.no_cpu, weights)

    small = small_64(not args.no_cpu)

    cpu = None
    if not args.no_cpu:
        log("[bench] timing the CPU oracle")
        cpu = cpu_baseline(job)
        log(f"[bench] oracle {cpu['value']:.3e} attempts/s on {cpu['cores']} threads")
        cpu["classical"] = classical_baseline()

    line = {
        "metric": "Kawasaki swap attempts/sec (4096^2 bit-packed lattice, omega=0.88, x=0.5)",
        "value": value, "unit": "attempts/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u1 (1 bit/site), int32 SWAR", "data": "synthetic",
        "config": {"workload": job.tag + f", {job.sweeps} sweeps + N_AB + cluster histogram per step",
                   "L": job.L, "composition": job.composition, "omega": job.omega,
                   "sweeps_per_step": job.sweeps, "layout": "bitpacked"},
        "roofline": roofline,
        "observables": {"ms": observe_ms, "similar_exact": obs["similar_exact"],
                        "similar_sampled": obs["similar_sampled"], "size_number_avg": obs["size_number_avg"],
                        "size_weight_avg": obs["size_weight_avg"]},
        "cpu_baseline": cpu,
        "small_64": small,
    }
    if batched is not None:
        line["batched"] = batched
        line["batched_offgrid"] = batched_off
    if grid is not None:
        line["grid_400"] = grid
    if served is not None:
        line["serving"] = served
    if tri is not None:
        line["triangular"] = tri
    if mp is not None:
        line["mpkk"] = mp
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
