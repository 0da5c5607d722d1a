"""Benchmark: accepted MH proposals/s of the tensor-network Metropolis-Hastings
chain on a 64x64 open ferromagnet at beta = 0.4407 with D = 32 environments,
4096 independent chains (one proposal per chain per step).

One step = one proposal per chain drawn by the batched fp32 MFMA sampler plus
the acceptance kernel.  The proposals do not depend on the chains' state, so
the sampler draws those of a few consecutive steps per launch; the chains are
bitwise those of one launch per step.  Before the timed region the library's
autotuner picks the sampler's launch variant and that step count by timing
them (all variants draw the same proposals).  The environment build (fp64
QR/SVD) is done once before the timed region and reported separately.  The plain fp64 GPU path (per-row
launches) runs the same chains from the same seeds for the comparison, and
the FP64 CPU oracle is timed on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "accepted MH proposals/s, 2D Ising L=64 D=32: batched FP32 vs plain FP64"
UNIT = "accepted proposals/s"
PEAK_FP32_MFMA = 157.3e12
PEAK_FP64_MFMA = 78.6e12
PEAK_BF16_MFMA = 2.5e15
PEAK_HBM = 8.0e12


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def tau_int(E, burn=0.1, c=6.0):
    """Integrated autocorrelation time of series E [steps, chains]: the
    correlation is averaged over chains and start times after a 10% burn-in,
    summed up to Sokal's window W >= 6 tau."""
    import numpy as np
    x = np.asarray(E, dtype=np.float64)
    x = x[int(burn * x.shape[0]):]
    n = x.shape[0]
    if n < 4:
        return float("nan")
    x = x - x.mean()
    var = (x * x).mean()
    if var == 0:
        return 1.0
    tau = 1.0
    for W in range(1, n):
        tau += 2.0 * (x[:-W] * x[W:]).mean() / var
        if W >= c * tau:
            break
    return float(tau)


def ahead_steps(chains):
    """MH steps whose proposals share one sampler launch: enough for two
    four-wave teams of 128 proposals per compute unit (proposals do not depend
    on the chains' state, Sec. 2, so drawing them ahead leaves the chains
    unchanged)."""
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    return max(1, -(-16 * 16 * cus // chains))


def run_gpu(prec, inst, steps, warmup, env_state=None, ahead=1, tune_steps=0, tune_cache=None):
    """tune_steps > 0: pick the sampler's launch variant and the MH steps per
    launch (up to tune_steps) with the library's autotuner before warm-up
    (tune_cache: its JSON file of earlier choices, or None); else variant 0
    and `ahead` steps per launch."""
    import numpy as np
    import torch
    from paper_2104_13264_amd import Sampler

    s = Sampler()
    t0 = time.perf_counter()
    if env_state is None:
        logZ = s.build_env(inst.Jh, inst.Jv, inst.h, inst.beta, inst.D, prec)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        env_state = s.get_env()
    else:
        env, dims, ell, logZ = env_state
        s.set_env(inst.Jh, inst.Jv, inst.h, inst.beta, inst.D, env, dims, ell, logZ, prec)
        build_s = None
    C = inst.chains
    variant = 0
    if tune_steps > 0:
        variant, ahead = s.autotune(C, max_steps=tune_steps, cache=tune_cache)
        log(f"[bench] tuned: variant {variant}, {ahead} MH steps per sampler launch")
    state = s.init_state(C)
    m = max(1, ahead)
    prop = (torch.empty((m, C, inst.Ly, inst.Lx), dtype=torch.int8, device=s.device),
            torch.empty((m, C), dtype=torch.float64, device=s.device),
            torch.empty((m, C), dtype=torch.float64, device=s.device))
    stream = torch.cuda.current_stream()

    def block(t, mm):
        out = (prop[0][:mm], prop[1][:mm], prop[2][:mm])
        s.sample_steps(C, mm, inst.seed, step0=t, out=out)

    def accept(t, j):
        s.mh_accept((prop[0][j], prop[1][j], prop[2][j]), state, inst.seed, t + j)

    t = 0
    while t < warmup:
        mm = min(m, warmup - t)
        block(t, mm)
        for j in range(mm):
            accept(t, j)
        t += mm
    s.stats(reset=True)
    E_series = torch.empty((steps, C), dtype=torch.float64, device=s.device)
    # the timed steps in launches of m steps, the remainder in a last launch
    launch_sizes = [m] * (steps // m) + ([steps % m] if steps % m else [])
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in launch_sizes]
    # the elementwise kernel that records the energy series runs once before
    # the timed region (its first launch loads the kernel)
    torch.mul(state["energy"], 1.0, out=E_series[0])
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    k = 0
    for li, mm in enumerate(launch_sizes):
        ev[li][0].record(stream)
        block(warmup + k, mm)
        ev[li][1].record(stream)
        for j in range(mm):
            accept(warmup + k, j)
            torch.mul(state["energy"], 1.0, out=E_series[k + j])   # an elementwise kernel, not a blit
        k += mm
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    kern_ms = [a.elapsed_time(b) for a, b in ev]
    for mm in sorted(set(launch_sizes), reverse=True):
        ms = [t for t, z in zip(kern_ms, launch_sizes) if z == mm]
        log(f"[bench] sampler launches of {mm} steps ({mm * C} proposals): {len(ms)} timed, "
            f"min {min(ms):.3f} median {float(np.median(ms)):.3f} max {max(ms):.3f} ms")
    st = s.stats()
    E = E_series.cpu().numpy()
    s.close()
    return dict(wall=wall, accepted=st["accepted"], proposed=st["proposed"],
                kern_ms=kern_ms, launch_sizes=launch_sizes,
                sampler_ms=float(np.mean(kern_ms)), steps_per_launch=m, variant=variant,
                build_s=build_s, logZ=logZ, E=E, near=st["near_threshold"],
                clamps=st["clamps"]), env_state


def run_cpu_oracle(inst, budget_s=12.0):
    """The oracle, as it stands, on a bounded sample of the same workload."""
    from oracle import bmps, ising, mh
    m = ising.Model(inst.Jh, inst.Jv, inst.h, inst.beta)
    envs = bmps.build_envs(m, inst.D)
    chains = 64
    state = mh.init_state(m, envs, chains)
    steps = 0
    acc_total = 0
    t0 = time.perf_counter()
    while True:
        acc, _, _ = mh.mh_step(m, envs, state, inst.seed, steps)
        acc_total += int(acc.sum())
        steps += 1
        if time.perf_counter() - t0 > budget_s or steps >= 50:
            break
    dt = time.perf_counter() - t0
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count()
    return dict(value=acc_total / dt, unit=UNIT, cores=cores, kind="oracle",
                sample=f"{steps} MH steps x {chains} chains of the 64x64 D=32 workload "
                       f"(numpy fp64, vectorised over chains, {dt:.1f} s); env build excluded",
                proposals_per_s=steps * chains / dt)


def run_ea_mix(steps, warmup):
    """64 uneven +-J instances: one MH step of all of them per captured graph
    replay (batched build, one sampler launch per bond class, one acceptance
    launch)."""
    import torch
    from paper_2104_13264_amd import Sampler, FP32
    from workloads import ea_mix, SEED
    insts = ea_mix()
    stream = torch.cuda.Stream()
    s = Sampler(stream=stream)
    t0 = time.perf_counter()
    lz = s.build_env_multi([dict(Jh=i.Jh, Jv=i.Jv, h=i.h, beta=i.beta, D=i.D, chains=i.chains)
                            for i in insts], FP32)
    build_s = time.perf_counter() - t0
    log(f"[bench] ea_mix: {len(insts)} environments built in {build_s:.2f} s")
    subs = [s.instance(k) for k in range(len(insts))]
    with torch.cuda.stream(stream):
        states = [sub.init_state(i.chains) for sub, i in zip(subs, insts)]
    stream.synchronize()
    variants = s.autotune_multi()   # launch variant of each bond class's sampler launch
    log(f"[bench] ea_mix: tuned variants {variants}")
    for t in range(warmup):
        s.mh_step_multi(states, SEED, t)
    stream.synchronize()
    for sub in subs:
        sub.stats(reset=True)
    t0 = time.perf_counter()
    s.graph_begin()
    s.mh_step_multi(states, SEED, warmup)
    s.graph_end_and_replay(steps)
    stream.synchronize()
    wall = time.perf_counter() - t0
    st = [sub.stats() for sub in subs]
    acc = sum(x["accepted"] for x in st)
    prop = sum(x["proposed"] for x in st)
    flops_step = sum(6.0 * i.D * i.D * i.Lx * i.Ly * i.chains for i in insts)
    by_L = {}
    for i, x in zip(insts, st):
        a = by_L.setdefault(i.Lx, [0, 0])
        a[0] += x["accepted"]
        a[1] += x["proposed"]
    s.close()
    return {"metric": "accepted MH proposals/s, 64 mixed +-J instances (batched, captured graph)",
            "value": acc / wall, "unit": UNIT, "n_gpus": 1, "steps": steps, "warmup": warmup,
            "ms_per_step": wall * 1e3 / steps, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
            "config": {"workload": "ea_mix: 64 Edwards-Anderson +-J instances, L in {16,24,32,48} "
                                   "(16 each), beta [1,2,3][i mod 3], D 16/32/32/64, 1024 chains "
                                   "each, one captured graph per MH step",
                       "sampler_variants": {f"{'bf16' if b else 'fp32'} D<={16 * nt}": v
                                            for (b, nt), v in sorted(variants.items())}},
            "acceptance": acc / max(prop, 1),
            "acceptance_by_L": {str(L): a[0] / max(a[1], 1) for L, a in sorted(by_L.items())},
            "achieved_tflops_6D2L2_minimum": flops_step * steps / wall / 1e12,
            "achieved_tflops_12D2L2": 2.0 * flops_step * steps / wall / 1e12,
            "env_build_s": build_s, "logZ_first": lz[0]}


def run_antiferro256(steps, warmup, n_eval=2048):
    """256x256 antiferromagnet, D = 64, BF16 operands with fp32 accumulation,
    16384 proposals per step; |ln q_BF16 - ln q_FP64| per sample on the drawn
    spins (fp64 eval of the same spins by the plain path)."""
    import numpy as np
    import torch
    from paper_2104_13264_amd import Sampler, FP64, FP32, BF16
    from workloads import antiferro_256
    inst = antiferro_256()
    s = Sampler()
    t0 = time.perf_counter()
    lz = s.build_env(inst.Jh, inst.Jv, inst.h, inst.beta, inst.D, BF16,
                     progress=lambda d, tot: log(f"[bench] env rows {d}/{tot} "
                                                 f"({time.perf_counter() - t0:.0f} s)"),
                     rows_per_call=24)
    build_s = time.perf_counter() - t0
    C = inst.chains
    out = {}
    for name, prec in (("bf16", BF16), ("fp32", FP32)):
        s.set_precision(prec)
        variant, _ = s.autotune(C, max_steps=1)   # launch variant of a one-step launch, timed
        log(f"[bench] antiferro256 {name}: tuned variant {variant}")
        state = s.init_state(C)
        prop = s.empty_batch(C)
        for t in range(warmup):
            s.sample(C, inst.seed, step=t, out=prop)
            s.mh_accept(prop, state, inst.seed, t)
        s.stats(reset=True)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        stream = torch.cuda.current_stream()
        t1 = time.perf_counter()
        for k in range(steps):
            ev[k][0].record(stream)
            s.sample(C, inst.seed, step=warmup + k, out=prop)
            ev[k][1].record(stream)
            s.mh_accept(prop, state, inst.seed, warmup + k)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t1
        st = s.stats()
        kms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
        out[name] = dict(value=st["accepted"] / wall, ms_per_step=wall * 1e3 / steps,
                         sampler_ms=kms, acceptance=st["accepted"] / max(st["proposed"], 1), variant=variant,
                         spins=prop[0][:n_eval].clone(), logq=prop[1][:n_eval].clone())
        log(f"[bench] antiferro256 {name}: {wall * 1e3 / steps:.1f} ms/step, sampler {kms:.1f} ms, "
            f"acceptance {out[name]['acceptance']:.4f}")
    # fp64 eval (plain path) of the last drawn spins of both paths
    s.set_precision(FP64)
    dev = {}
    for name in ("bf16", "fp32"):
        lq64, _ = s.eval_logq(out[name]["spins"])
        d = (out[name]["logq"] - lq64).abs().cpu().numpy()
        dev[name] = dict(max=float(d.max()), mean=float(d.mean()),
                         rel_max=float((d / lq64.abs().cpu().numpy()).max()))
    s.close()
    flops = 12.0 * inst.D ** 2 * inst.Lx * inst.Ly * C   # the method's count per proposal, 12 D^2 L^2
    return {"metric": "accepted MH proposals/s, 2D Ising L=256 D=64: batched BF16 (and FP32)",
            "value": out["bf16"]["value"], "unit": UNIT, "n_gpus": 1, "steps": steps,
            "warmup": warmup, "ms_per_step": out["bf16"]["ms_per_step"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
            "config": {"workload": "antiferro256_D64: 256x256 open antiferromagnet J=-1, h=0, "
                                   "beta=0.4407, D=64 (fp64 build), 16384 chains from all-up"},
            "acceptance": out["bf16"]["acceptance"],
            "roofline": {"bound": "mfma", "achieved": flops / (out["bf16"]["sampler_ms"] * 1e-3) / 1e12,
                         "peak": 2500.0, "unit": "TFLOP/s",
                         "frac": flops / (out["bf16"]["sampler_ms"] * 1e-3) / 2.5e15,
                         "traffic": measured_traffic(C, out["bf16"]["variant"], "sampler_team_antiferro256_traffic.json"),
                         "kernel": f"k_sampler_team<4,1,{out['bf16']['variant']}>",
                         "flop_count": "12 D^2 L^2 per proposal",
                         "frac_6D2L2_minimum": flops / 2 / (out["bf16"]["sampler_ms"] * 1e-3) / 2.5e15,
                         "kernel_ms": out["bf16"]["sampler_ms"]},
            "fp32": {k: v for k, v in out["fp32"].items() if k not in ("spins", "logq")},
            "abs_logq_minus_fp64": dev, "n_eval": n_eval,
            "env_build_s": build_s, "logZ": lz}


def run_peaks(reps=3):
    """Attained peak of each unit the kernels use (tn_peak_probe): the best of
    `reps` timed launches per probe, beside the published figure; for the
    arithmetic probes also the clock that the rate implies (rate over the
    chip's flops per cycle: 256 CUs x 4 SIMDs x the unit's flops per SIMD and
    cycle)."""
    from paper_2104_13264_amd import peak_probe
    probes = [  # kind, amount, published peak, unit scale, flops per cycle of the chip
        ("mfma_f32", 60000, PEAK_FP32_MFMA, 1e12, 1024 * 64),
        ("mfma_bf16", 120000, PEAK_BF16_MFMA, 1e12, 1024 * 1024),
        ("mfma_f64", 30000, PEAK_FP64_MFMA, 1e12, 1024 * 32),
        ("fma_f64", 200000, PEAK_FP64_MFMA, 1e12, 1024 * 32),
        ("hbm_read", 16 << 30, PEAK_HBM, 1e9, None),
        ("hbm_copy", 8 << 30, PEAK_HBM, 1e9, None),
    ]
    out = {}
    for kind, amount, peak, scale, per_cycle in probes:
        best = 0.0
        for _ in range(reps):
            sec, work = peak_probe(kind, amount)
            best = max(best, work / sec)
        e = {"attained": best / scale, "published": peak / scale,
             "unit": "TFLOP/s" if per_cycle else "GB/s", "frac": best / peak}
        if per_cycle:
            e["implied_clock_ghz"] = best / per_cycle / 1e9
        log(f"[bench] peak {kind}: {e['attained']:.1f} {e['unit']} of {e['published']:.1f} "
            f"({100 * e['frac']:.1f}%)" + (f", implied clock {e['implied_clock_ghz']:.2f} GHz" if per_cycle else ""))
        out[kind] = e
    return {"metric": "attained peak per unit (one unit alone, best of %d launches)" % reps, "probes": out,
            "n_gpus": 1, "data": "synthetic"}


def run_potts(steps, warmup, L=32, d=3, D=16, chains=8192):
    """q-state Potts ferromagnet (general local dimension d, App. A), L x L
    open boundaries, J = 1, h = 0, at the critical coupling of the square
    lattice, beta = ln(1 + sqrt(d)); plain fp64 sampler with d-way
    conditionals, one MH step of `chains` chains per step from all value 0.
    The roofline is that of the row-sampler kernel (fp64 vector work): per
    site the environment sweep's d products with D x D matrices, the drawing
    product and the d weights, (d + 1) 2 D^2 + 2 d D flops."""
    import math
    import numpy as np
    import torch
    from paper_2104_13264_amd import Sampler
    from workloads import SEED
    beta = math.log(1.0 + math.sqrt(d))
    Jh, Jv = np.ones((L, L - 1)), np.ones((L - 1, L))
    s = Sampler()
    t0 = time.perf_counter()
    lz = s.potts_build_env(Jh, Jv, None, beta, D, d)
    build_s = time.perf_counter() - t0
    log(f"[bench] potts {L}x{L} d={d} D={D}: build {build_s:.2f} s, ln Z~ {lz:.6f}")
    state = s.init_state(chains)
    prop = s.empty_batch(chains)
    for t in range(warmup):
        s.sample(chains, SEED, step=t, out=prop)
        s.mh_accept(prop, state, SEED, t)
    s.stats(reset=True)
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    E_series = torch.empty((steps, chains), dtype=torch.float64, device=s.device)
    torch.mul(state["energy"], 1.0, out=E_series[0])   # loads the kernel before the timed region
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record(stream)
        s.sample(chains, SEED, step=warmup + k, out=prop)
        ev[k][1].record(stream)
        s.mh_accept(prop, state, SEED, warmup + k)
        torch.mul(state["energy"], 1.0, out=E_series[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    st = s.stats()
    kms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    s.close()
    flops = ((d + 1) * 2.0 * D * D + 2.0 * d * D) * L * L * chains
    achieved = flops / (kms * 1e-3)
    # the oracle on the host cores, a bounded sample of the same workload
    from oracle import potts as opotts
    m = opotts.PottsModel(Jh, Jv, None, beta, d)
    envs = opotts.build_envs(m, D)
    ost = opotts.init_state(m, envs, 64)
    n, acc_o, tc = 0, 0, time.perf_counter()
    while n < 20 and time.perf_counter() - tc < 10.0:
        acc_o += int(opotts.mh_step(m, envs, ost, SEED, n).sum())
        n += 1
    dt = time.perf_counter() - tc
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count()
    return {"metric": "accepted MH proposals/s, 3-state Potts L=32 D=16 at beta_c: plain FP64 (d-way draw)",
            "value": st["accepted"] / wall, "unit": UNIT, "n_gpus": 1, "steps": steps, "warmup": warmup,
            "ms_per_step": wall * 1e3 / steps, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"potts{d}_{L}x{L}_D{D}: {d}-state Potts ferromagnet J=1, h=0, "
                                   f"beta=ln(1+sqrt({d}))={beta:.6f}, open boundaries, {chains} chains "
                                   "from all value 0, one proposal per chain per step"},
            "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": 78.6, "unit": "TFLOP/s",
                         "frac": achieved / 78.6e12, "traffic": None,
                         "kernel": f"k_potts_rows<{1 << (D - 1).bit_length()},{d}> (one launch per row)",
                         "flop_count": "((d+1) 2 D^2 + 2 d D) L^2 per proposal",
                         "kernel_ms_per_step": kms},
            "acceptance": st["accepted"] / max(st["proposed"], 1),
            "tau_int_mean_energy": tau_int(E_series.cpu().numpy()),
            "near_threshold_draws": st["near_threshold"], "clamps": st["clamps"],
            "env_build_s": build_s, "logZ": lz,
            "cpu_baseline": {"value": acc_o / dt, "unit": UNIT, "cores": cores, "kind": "oracle",
                             "sample": f"{n} MH steps x 64 chains of the same workload (numpy fp64, {dt:.1f} s)"}}


def run_hybrid(steps=200, chains=1024, sweeps=1):
    """+-J spin glass 32x32 at T = 0.212 (beta = 4.717) with D = 16, the
    temperature, size and bond dimension of the paper's interleaving
    experiment (Fig. hb b), FP32: TNMH steps alone and with one
    single-spin-flip Metropolis sweep after each step, from all-up, same
    seeds.  Reports the acceptance, the energy reached and the cost of a sweep
    call (sweep kernel plus the re-evaluation of ln q)."""
    import numpy as np
    import torch
    from paper_2104_13264_amd import Sampler, FP32
    from workloads import ea_pm, SEED
    inst = ea_pm(32, 1.0 / 0.212, 16, SEED + 7, chains=chains)
    s = Sampler()
    t0 = time.perf_counter()
    s.build_env(inst.Jh, inst.Jv, None, inst.beta, inst.D, FP32)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    degen = s.stats()["degenerate_cuts"]   # truncations at tied singular values
    out = {"workload": "hybrid_ea32_T0.212_D16", "chains": chains, "steps": steps, "env_build_s": build_s,
           "logZ": s.stats()["logZ"]}
    stream = torch.cuda.current_stream()
    for mode in ("tnmh", "tnmh+metropolis"):
        state = s.init_state(chains)
        s.stats(reset=True)
        E = np.zeros(steps)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(steps):
            s.mh_step(state, SEED, t)
            if mode != "tnmh":
                ev[2 * t].record(stream)
                s.metropolis_sweeps(state, sweeps, SEED, t)
                ev[2 * t + 1].record(stream)
            E[t] = float(state["energy"].mean())
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = s.stats()
        r = {"acceptance": st["accepted"] / max(st["proposed"], 1), "ms_per_step": wall * 1e3 / steps,
             "mean_energy_per_site_last_quarter": float(E[3 * steps // 4:].mean()) / (inst.Lx * inst.Ly),
             "energy_per_site_at": {str(t): E[t] / (inst.Lx * inst.Ly) for t in (0, 9, 49, steps - 1)}}
        if mode != "tnmh":
            call_ms = [ev[2 * t].elapsed_time(ev[2 * t + 1]) for t in range(steps)]
            r["sweep_call_ms"] = float(np.median(call_ms))
            r["flips_per_site_update"] = st["metropolis_flips"] / (steps * sweeps * chains * inst.Lx * inst.Ly)
        out[mode] = r
        log(f"[bench] hybrid {mode}: acceptance {r['acceptance']:.4f}, E/site last quarter "
            f"{r['mean_energy_per_site_last_quarter']:.5f}, {r['ms_per_step']:.2f} ms/step")
    # the sweep call is the sweep kernel plus ln q of the new states; time the
    # latter alone to split them
    state = s.init_state(chains)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(5):
        s.eval_logq(state["spins"])
    e1.record(stream)
    torch.cuda.synchronize()
    eval_ms = e0.elapsed_time(e1) / 5
    kern_ms = out["tnmh+metropolis"]["sweep_call_ms"] - eval_ms
    out["eval_logq_ms"] = eval_ms
    out["sweep_kernel_ms_est"] = kern_ms
    out["site_updates_per_s_est"] = sweeps * chains * inst.Lx * inst.Ly / (kern_ms * 1e-3) if kern_ms > 0 else None
    # the same environments with FP64 operands (plain path): how much of the
    # FP32 acceptance is lost to the rounding of ln q
    from paper_2104_13264_amd import FP64
    s.set_precision(FP64)
    state = s.init_state(chains)
    s.stats(reset=True)
    n64 = 60
    for t in range(n64):
        s.mh_step(state, SEED, t)
    st = s.stats()
    out["fp64_acceptance_60_steps"] = st["accepted"] / max(st["proposed"], 1)
    out["degenerate_cuts"] = degen
    log(f"[bench] hybrid tnmh, FP64 operands: acceptance {out['fp64_acceptance_60_steps']:.5f} over {n64} steps")
    s.close()
    return out


def run_fitbuild(sweeps=(0, 1, 2), n_inst=64):
    """Batched environment builds of the 64 Gaussian 32x32 instances of the
    delta workload (T = 0.212, D = 16) by successive SVD and with 1 and 2
    two-site variational sweeps per row: wall time and ln Z~ of instance 0."""
    import torch
    from paper_2104_13264_amd import Sampler, FP32
    from workloads import ea_gauss_set
    insts = ea_gauss_set(n=n_inst, chains=30)
    out = {"workload": "fitbuild_ea_gauss32_T0.212_D16", "instances": n_inst, "rows": []}
    for sw in sweeps:
        s = Sampler()
        s.set_compression(sw)
        dicts = [dict(Jh=i.Jh, Jv=i.Jv, h=None, beta=i.beta, D=i.D, chains=i.chains) for i in insts]
        s.build_env_multi(dicts, FP32)   # first build allocates
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lz = s.build_env_multi(dicts, FP32)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s.close()
        out["rows"].append({"fit_sweeps": sw, "build_s": dt, "logZ_0": lz[0]})
        log(f"[bench] fitbuild: {sw} sweeps, {n_inst} builds in {dt:.3f} s, ln Z~[0] = {lz[0]:.9f}")
    return out


def run_precision(steps=40, chains=1024, temps=(1.0, 0.5, 0.3, 0.212)):
    """Acceptance of the sampler precisions on one environment build: the
    +-J 32x32 instance of the hybrid workload, D = 16, from all-up, at several
    temperatures (FP64 plain path; FP64, FP32 and BF16 operands on the batched
    path; the operands of each are derived from the same FP64 environments)."""
    import torch
    from paper_2104_13264_amd import Sampler, FP64, FP32, BF16, FP64_MFMA
    from workloads import ea_pm, SEED
    out = {"workload": "precision_ea32_D16", "chains": chains, "steps": steps, "rows": []}
    for T in temps:
        inst = ea_pm(32, 1.0 / T, 16, SEED + 7, chains=chains)
        s = Sampler()
        s.build_env(inst.Jh, inst.Jv, None, inst.beta, 16, FP64)
        row = {"T": T, "degenerate_cuts": s.stats()["degenerate_cuts"]}
        for name, prec in (("fp64", FP64), ("fp64_mfma", FP64_MFMA), ("fp32", FP32), ("bf16", BF16)):
            s.set_precision(prec)
            state = s.init_state(chains)
            s.stats(reset=True)
            for t in range(steps):
                s.mh_step(state, SEED, t)
            st = s.stats()
            row[name] = st["accepted"] / max(st["proposed"], 1)
        torch.cuda.synchronize()
        s.close()
        out["rows"].append(row)
        log(f"[bench] precision T={T}: acceptance fp64 {row['fp64']:.5f}, fp64_mfma {row['fp64_mfma']:.5f}, "
            f"fp32 {row['fp32']:.5f}, "
            f"bf16 {row['bf16']:.5f} (degenerate cuts {row['degenerate_cuts']})")
    return out


def run_delta(steps=40, n_inst=64, chains=30, prec=None, modes=(("tnmh", 0), ("tnmh+metropolis", 1)),
              fit_sweeps=0):
    """Equilibration test of Sec. 3, Eq. (Delta), on Gaussian spin glasses in
    the setting of the paper's Fig. hb b: n_inst 32x32 open instances at
    T = 0.212, D = 16, 30 chains each (15 replica pairs), from uniform random
    configurations; MH steps of all instances together (`modes`: name and
    Metropolis sweeps after each step).  Delta(t) is the disorder average
    over the instances of <H>/|V| + beta (|E| - link overlap)/|V| with the
    thermal averages over each instance's chains and replica pairs.
    fit_sweeps > 0: environments by successive SVD and that many two-site
    variational sweeps (the compression App. A names for these runs)."""
    import numpy as np
    import torch
    from paper_2104_13264_amd import Sampler, FP32
    from workloads import ea_gauss_set, random_spins, SEED
    prec = FP32 if prec is None else prec
    insts = ea_gauss_set(n=n_inst, chains=chains)
    L = insts[0].Lx
    nV, nE = L * L, 2 * L * (L - 1)
    beta = insts[0].beta
    s = Sampler()
    s.set_compression(fit_sweeps)
    t0 = time.perf_counter()
    s.build_env_multi([dict(Jh=i.Jh, Jv=i.Jv, h=None, beta=i.beta, D=i.D, chains=i.chains) for i in insts], prec)
    build_s = time.perf_counter() - t0
    log(f"[bench] delta: {n_inst} Gaussian instances built in {build_s:.2f} s")
    subs = [s.instance(k) for k in range(n_inst)]
    out = {"workload": "delta_ea_gauss32_T0.212_D16", "instances": n_inst, "chains": chains,
           "steps": steps, "env_build_s": build_s, "fit_sweeps": fit_sweeps}
    thresholds = (0.25, 0.15, 0.05, 0.025)
    for mode, nsw in modes:
        states = [sub.init_state(chains, torch.as_tensor(random_spins(chains, L, L, SEED + 77 + k)))
                  for k, sub in enumerate(subs)]
        for sub in subs:
            sub.stats(reset=True)

        def delta_now():
            d = []
            for sub, st in zip(subs, states):
                e = float(st["energy"].mean())
                q = float(sub.link_overlap(st["spins"][0::2], st["spins"][1::2]).double().mean())
                d.append(e / nV + beta * (nE - q) / nV)
            return float(np.mean(d))

        series = [delta_now()]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for t in range(steps):
            s.mh_step_multi(states, SEED, t)
            if nsw:
                for sub, st in zip(subs, states):
                    sub.metropolis_sweeps(st, nsw, SEED, t)
            series.append(delta_now())
        torch.cuda.synchronize()
        wall = time.perf_counter() - t1
        acc = sum(sub.stats()["accepted"] for sub in subs)
        prop = sum(sub.stats()["proposed"] for sub in subs)
        first = {str(th): next((t for t, v in enumerate(series) if v < th), None) for th in thresholds}
        out[mode] = {"delta": series, "steps_to_reach": first, "acceptance": acc / max(prop, 1),
                     "ms_per_step": wall * 1e3 / steps}
        log(f"[bench] delta {mode}: Delta(0) {series[0]:.3f}, Delta({steps}) {series[-1]:.4f}, "
            f"steps to reach {first}, acceptance {acc / max(prop, 1):.4f}")
    s.close()
    return out


def run_periodic(steps=60, n_inst=64, chains=30, D=16, prec=None, cuts="random", sweeps=0):
    """Equilibration test of Eq. (Delta) with periodic boundaries (Section
    "Arbitrary boundary conditions", table of TNMH iterations on periodic
    Gaussian spin glasses): n_inst 32x32 tori at T = 0.212, D = 16, 30 chains
    each (15 replica pairs) from uniform random configurations; every step
    freezes a cross (row and column) drawn uniformly at random, builds every
    chain's open model and takes one TNMH step per chain.  Delta(t) as in
    run_delta with the 2 L^2 bonds of the torus.  cuts: "opposite" alternates
    between two opposite crosses, (k, k) and (k + L/2, k + L/2) with k = t // 2
    (the torus analogue of the paper's alternating opposite lines, shifted so
    that no site stays frozen), "random" draws a uniform cross per step.
    sweeps: Metropolis sweeps on the torus after every TNMH step."""
    import numpy as np
    import torch
    from paper_2104_13264_amd import Sampler, FP32
    from workloads import ea_gauss_torus_set, random_spins, SEED
    prec = FP32 if prec is None else prec
    insts = ea_gauss_torus_set(n=n_inst, chains=chains)
    L = insts[0]["Jh"].shape[0]
    nV, nE = L * L, 2 * L * L
    beta = insts[0]["beta"]
    s = Sampler()
    t0 = time.perf_counter()
    s.periodic_setup(insts, L, L, True, True, D, prec)
    setup_s = time.perf_counter() - t0
    T = n_inst * chains
    spins = torch.as_tensor(np.concatenate([random_spins(chains, L, L, SEED + 77 + k) for k in range(n_inst)]),
                            device=s.device).contiguous()
    E = s.periodic_energy(spins)
    if cuts == "random":
        cut = np.random.default_rng(SEED + 5).integers(0, L, size=(steps, 2))
    else:
        k = np.arange(steps) // 2 + (np.arange(steps) % 2) * (L // 2)
        cut = np.stack([k % L, k % L], axis=1)
    log(f"[bench] periodic: {n_inst} tori x {chains} chains set up in {setup_s:.2f} s")

    def delta_now(E):
        q = s.periodic_link_overlap(spins[0::2], spins[1::2]).double().view(n_inst, chains // 2).mean(1)
        e = E.view(n_inst, chains).mean(1)
        return float((e / nV + beta * (nE - q) / nV).mean())

    series = [delta_now(E)]
    s.stats(reset=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_ms = []
    for t in range(steps):
        ts = time.perf_counter()
        E, acc = s.periodic_step(spins, SEED, t, int(cut[t, 0]), int(cut[t, 1]))
        if sweeps:
            E = s.periodic_sweeps(spins, sweeps, SEED, t)
        torch.cuda.synchronize()
        step_ms.append((time.perf_counter() - ts) * 1e3)
        series.append(delta_now(E))
        if t % 10 == 9:
            log(f"[bench] periodic step {t + 1}: Delta {series[-1]:.4f}")
    wall = time.perf_counter() - t1
    st = s.stats()
    thresholds = (0.25, 0.15, 0.05, 0.025)
    first = {str(th): next((t for t, v in enumerate(series) if v < th), None) for th in thresholds}
    s.close()
    out = {"workload": f"periodic_ea_gauss_torus{L}_T0.212_D{D}", "instances": n_inst, "chains": chains,
           "chains_total": T, "steps": steps, "setup_s": setup_s,
           "cuts": "uniform random cross per step" if cuts == "random" else "alternating opposite crosses",
           "metropolis_sweeps_per_step": sweeps,
           "delta": series, "steps_to_reach": first,
           "acceptance": st["accepted"] / max(st["proposed"], 1),
           "ms_per_step": wall * 1e3 / steps, "ms_per_step_median": float(np.median(step_ms)),
           "chain_steps_per_s": T * steps / wall}
    log(f"[bench] periodic: Delta(0) {series[0]:.3f}, Delta({steps}) {series[-1]:.4f}, steps to reach {first}, "
        f"acceptance {out['acceptance']:.4f}, {out['ms_per_step']:.1f} ms per step")
    return out


def run_frustrated128(chains=1024, steps=60, warmup=20, bonds=8, fd_bonds=2):
    """128x128 fully frustrated lattice, beta = 1, D = 32: d ln Z~ / dJ and
    d ln Z~ / d beta (tn_grad), timed, beside the chain's own estimates of
    beta <s_i s_j> on a few bonds and of -<E>."""
    import numpy as np
    import torch
    from paper_2104_13264_amd import Sampler, FP32
    from workloads import frustrated_128, SEED
    inst = frustrated_128()
    s = Sampler()
    t0 = time.perf_counter()
    lz = s.build_env(inst.Jh, inst.Jv, inst.h, inst.beta, inst.D, FP32,
                     progress=lambda d, tot: log(f"[bench] env rows {d}/{tot}"), rows_per_call=32)
    build_s = time.perf_counter() - t0
    t1 = time.perf_counter()
    dJh, dJv, db = s.grad()
    torch.cuda.synchronize()
    grad_s = time.perf_counter() - t1
    log(f"[bench] frustrated128: build {build_s:.1f} s, gradient {grad_s:.1f} s")
    t1 = time.perf_counter()
    tJh, tJv, tdb = s.grad(two_sided=True)
    torch.cuda.synchronize()
    two_s = time.perf_counter() - t1
    log(f"[bench] frustrated128: two-sided estimate {two_s:.1f} s (with the upside-down build)")
    state = s.init_state(chains)
    rng = np.random.default_rng(SEED)
    pick = [(int(rng.integers(0, 128)), int(rng.integers(0, 127))) for _ in range(bonds)]
    corr = [[] for _ in range(bonds)]
    en = []
    for t in range(warmup + steps):
        s.mh_step(state, SEED, t)
        if t >= warmup:
            sp = state["spins"].double()
            for k, (r, c) in enumerate(pick):
                corr[k].append(float((sp[:, r, c] * sp[:, r, c + 1]).mean()))
            en.append(float(state["energy"].mean()))
    st = s.stats()
    g = dJh.cpu().numpy()
    g2 = tJh.cpu().numpy()
    # central differences of the rebuilt ln Z~ (truncations free to move) on
    # the first fd_bonds bonds, step 1e-4
    fd = []
    for k, (r, c) in enumerate(pick[:fd_bonds]):
        vals = []
        for sgn in (1.0, -1.0):
            Jh = inst.Jh.copy()
            Jh[r, c] += sgn * 1e-4
            vals.append(s.build_env(Jh, inst.Jv, inst.h, inst.beta, inst.D, FP32))
        fd.append((vals[0] - vals[1]) / 2e-4)
        log(f"[bench] frustrated128: finite difference {k + 1}/{fd_bonds}")
    s.close()
    err = lambda xs: float(np.std(xs) / np.sqrt(len(xs)))
    return {"workload": "frustrated128_D32", "env_build_s": build_s, "grad_s": grad_s, "logZ": lz,
            "dlogZ_dbeta": db, "chain_minus_mean_energy": -float(np.mean(en)),
            "chain_minus_mean_energy_err": err(en),
            "bonds": pick, "grad_dJh": [float(g[r, c]) for r, c in pick],
            "chain_beta_corr": [float(inst.beta * np.mean(x)) for x in corr],
            "chain_beta_corr_err": [inst.beta * err(x) for x in corr],
            "fd_dJh": fd, "grad_finite": bool(np.isfinite(g).all()),
            "two_sided_s": two_s, "two_sided_dJh": [float(g2[r, c]) for r, c in pick],
            "two_sided_dlogZ_dbeta": tdb,
            "acceptance": st["accepted"] / max(st["proposed"], 1), "chains": chains, "steps": steps}


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ["sampler_mfma.hip", "operands.hip", "common.hpp"]:
        with open(os.path.join(ROOT, "paper_2104_13264_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(proposals_per_launch, variant, name="sampler_team_ferro64_traffic.json"):
    """HBM bytes per sampler launch from committed rocprofv3 counter runs, if
    they were taken on the current kernel source in this launch shape (the
    file holds one entry per measured shape)."""
    p = os.path.join(ROOT, "profiles", name)
    try:
        with open(p) as fh:
            d = json.load(fh)
    except OSError:
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    for e in d.get("entries", []):
        if e.get("proposals_per_launch") == proposals_per_launch and e.get("variant", 0) == variant:
            return e.get("bytes_per_launch")
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain fp64 path")
    ap.add_argument("--no-batched-fp64", action="store_true",
                    help="skip the batched fp64 path (fp64 operands on the matrix cores)")
    ap.add_argument("--no-batched-bf16", action="store_true",
                    help="skip the batched bf16 path (bf16 operands, fp32 accumulation)")
    ap.add_argument("--tune-steps", type=int, default=32,
                    help="largest MH-step count per sampler launch the autotuner tries "
                         "(0: no tuning, variant 0 and the built-in count)")
    ap.add_argument("--tune-cache", default=None,
                    help="the autotuner's JSON file of earlier choices (default: time afresh)")
    ap.add_argument("--force-variant", type=int, default=None,
                    help="batched FP32 leg: use this launch variant with launches of all the timed steps "
                         "(through a tuning-cache entry; for counter runs of other launch shapes)")
    ap.add_argument("--ahead", type=int, default=None,
                    help="MH steps per sampler launch (default: enough for two four-wave teams per CU)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 256 MiB device-to-device copy (counter calibration)")
    ap.add_argument("--fit-sweeps", type=int, default=0,
                    help="delta workload: also run with this many two-site variational sweeps")
    ap.add_argument("--periodic-steps", type=int, default=60,
                    help="TNMH steps of the periodic workload")
    ap.add_argument("--periodic-sweeps", type=int, default=0,
                    help="Metropolis sweeps after every TNMH step of the periodic workload")
    ap.add_argument("--periodic-cuts", default="random", choices=["random", "opposite"],
                    help="cut schedule of the periodic workload")
    ap.add_argument("--workload", default="ferro64",
                    choices=["ferro64", "ea_mix", "antiferro256", "frustrated128", "hybrid", "delta",
                             "periodic", "precision", "fitbuild", "potts", "peaks"],
                    help="ferro64 is the headline line; the others report the other workloads")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the sampler "
              "shards by chains, one process per GPU, and only one GPU is measured here", file=sys.stderr)
        sys.exit(2)
    if args.calib_copy:
        # a plain copy of known size for counter calibration: 256 MiB read + 256 MiB written
        import torch
        x = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    if args.workload != "ferro64":
        if args.workload == "ea_mix":
            out = run_ea_mix(args.steps, args.warmup)
        elif args.workload == "antiferro256":
            out = run_antiferro256(min(args.steps, 20), min(args.warmup, 2))
        elif args.workload == "hybrid":
            out = run_hybrid()
        elif args.workload == "delta":
            from paper_2104_13264_amd import FP64, FP32
            out = {"fp32": run_delta(prec=FP32), "fp64": run_delta(prec=FP64)}
            if args.fit_sweeps:
                out["fp32_fit"] = run_delta(prec=FP32, fit_sweeps=args.fit_sweeps, modes=(("tnmh", 0),))
                out["fp64_fit"] = run_delta(prec=FP64, fit_sweeps=args.fit_sweeps)
        elif args.workload == "fitbuild":
            out = run_fitbuild()
        elif args.workload == "precision":
            out = run_precision()
        elif args.workload == "potts":
            out = run_potts(args.steps, args.warmup)
        elif args.workload == "peaks":
            out = run_peaks()
        elif args.workload == "periodic":
            out = run_periodic(steps=args.periodic_steps, cuts=args.periodic_cuts, sweeps=args.periodic_sweeps)
        else:
            out = run_frustrated128()
        print(json.dumps(out), flush=True)
        return
    import numpy as np
    import torch
    from workloads import ferro_64

    inst = ferro_64()
    L, D, C = inst.Lx, inst.D, inst.chains
    log(f"[bench] ferro 64x64 D={D} chains={C} steps={args.steps} warmup={args.warmup}")

    m = ahead_steps(C) if args.ahead is None else args.ahead
    tune_cache = args.tune_cache
    if args.force_variant is not None:
        # a cache entry the tuner takes as found: the variant, and launches of
        # all the timed steps
        import tempfile
        import torch
        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
        steps = min(args.tune_steps, args.steps)
        key = f"{arch}|{L}x{inst.Ly}|D{D}|fp32|chains{C}|steps{steps}"
        tune_cache = os.path.join(tempfile.mkdtemp(), "forced.json")
        with open(tune_cache, "w") as fh:
            fh.write("{\n  " + json.dumps(key) + ": " +
                     json.dumps({"variant": args.force_variant, "proposals": steps * C, "ns_per_proposal": 0.0}) + "\n}\n")
    res32, env_state = run_gpu(1, inst, args.steps, args.warmup, ahead=m,
                               tune_steps=0 if args.ahead is not None else min(args.tune_steps, args.steps),
                               tune_cache=tune_cache)
    m = res32["steps_per_launch"]
    log(f"[bench] fp32 batched: {res32['wall']*1e3/args.steps:.3f} ms/step, "
        f"sampler launches of {res32['launch_sizes']} steps: {sum(res32['kern_ms']):.3f} ms in total, "
        f"acc {res32['accepted']}/{res32['proposed']}, env build {res32['build_s']:.2f} s")
    res64 = None
    if not args.no_plain:
        res64, _ = run_gpu(0, inst, args.steps, args.warmup, env_state)
        log(f"[bench] fp64 plain: {res64['wall']*1e3/args.steps:.3f} ms/step, "
            f"acc {res64['accepted']}/{res64['proposed']}")

    res64m = None
    if not args.no_batched_fp64:
        res64m, _ = run_gpu(3, inst, args.steps, args.warmup, env_state,
                            ahead=m, tune_steps=0 if args.ahead is not None else min(args.tune_steps, args.steps),
                            tune_cache=args.tune_cache)
        log(f"[bench] fp64 batched: {res64m['wall']*1e3/args.steps:.3f} ms/step, "
            f"sampler launches of {res64m['launch_sizes']} steps: {sum(res64m['kern_ms']):.3f} ms in total, "
            f"acc {res64m['accepted']}/{res64m['proposed']}")

    res16 = None
    if not args.no_batched_bf16:
        res16, _ = run_gpu(2, inst, args.steps, args.warmup, env_state,
                           ahead=m, tune_steps=0 if args.ahead is not None else min(args.tune_steps, args.steps),
                           tune_cache=args.tune_cache)
        log(f"[bench] bf16 batched: {res16['wall']*1e3/args.steps:.3f} ms/step, variant {res16['variant']}, "
            f"sampler launches of {res16['launch_sizes']} steps: {sum(res16['kern_ms']):.3f} ms in total, "
            f"acc {res16['accepted']}/{res16['proposed']}")

    value = res32["accepted"] / res32["wall"]
    ms_per_step = res32["wall"] * 1e3 / args.steps
    # Roofline of the sampler launches timed above (HIP events on the stream
    # they run on), from the proposals they actually drew.  Algorithmic work
    # per proposal, three counts:
    #   12 D^2 L^2  the method's count: per site, the right environment with
    #               its horizontal leg (8 D^2) and the drawing product (4 D^2)
    #    6 D^2 L^2  the minimum: the horizontal bond contracted exactly, both
    #               spins' right products (4 D^2) and the drawn spin's left
    #               product (2 D^2)
    #    8 D^2 L^2  what the kernel executes: both spins' left products
    props = C * sum(res32["launch_sizes"])
    kern_s = sum(res32["kern_ms"]) * 1e-3
    flops = {k: f * D * D * L * L * props for k, f in (("12D2L2", 12.0), ("6D2L2", 6.0), ("8D2L2", 8.0))}
    achieved = flops["12D2L2"] / kern_s
    shapes = sorted(set(res32["launch_sizes"]))
    traffic = measured_traffic(C * shapes[0], res32["variant"]) if len(shapes) == 1 else None
    out = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": "ferro64_D32: 64x64 open-boundary ferromagnet J=+1, h=0, "
                               "beta=0.4407, D=32 fp64 environments, 4096 chains from all-up, "
                               "one proposal per chain per step",
                   "chains": C, "L": L, "D": D, "beta": inst.beta, "seed": inst.seed,
                   "mh_steps_per_sampler_launch": res32["steps_per_launch"],
                   "sampler_variant": res32["variant"]},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_FP32_MFMA / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_MFMA,
                     "traffic": traffic,
                     "kernel": f"k_sampler_team<2,0,{res32['variant']}>",
                     "flop_count": "12 D^2 L^2 per proposal",
                     "frac_6D2L2_minimum": flops["6D2L2"] / kern_s / PEAK_FP32_MFMA,
                     "frac_8D2L2_executed": flops["8D2L2"] / kern_s / PEAK_FP32_MFMA,
                     "launch_steps": res32["launch_sizes"],
                     "proposals_timed": props,
                     "kernel_ms_total": sum(res32["kern_ms"]),
                     "kernel_ms": res32["sampler_ms"]},
        "acceptance": res32["accepted"] / max(res32["proposed"], 1),
        "proposals_per_s": res32["proposed"] / res32["wall"],
        "tau_int_mean_energy": tau_int(res32["E"]),
        "env_build_s": res32["build_s"],
        "logZ": res32["logZ"],
        "near_threshold_draws": res32["near"],
    }
    if res64 is not None:
        v64 = res64["accepted"] / res64["wall"]
        out["plain_fp64"] = {"value": v64, "unit": UNIT,
                             "ms_per_step": res64["wall"] * 1e3 / args.steps,
                             "acceptance": res64["accepted"] / max(res64["proposed"], 1),
                             "tau_int_mean_energy": tau_int(res64["E"]),
                             "sampler_ms": res64["sampler_ms"]}
        out["speedup_vs_plain_fp64"] = value / v64 if v64 > 0 else None
    if res64m is not None:
        v64m = res64m["accepted"] / res64m["wall"]
        props64 = C * sum(res64m["launch_sizes"])
        kern64 = sum(res64m["kern_ms"]) * 1e-3
        out["batched_fp64"] = {"value": v64m, "unit": UNIT,
                               "ms_per_step": res64m["wall"] * 1e3 / args.steps,
                               "acceptance": res64m["accepted"] / max(res64m["proposed"], 1),
                               "tau_int_mean_energy": tau_int(res64m["E"]),
                               "kernel": f"k_sampler_team<{-(-D // 16)},2,{res64m['variant']}>",
                               "launch_steps": res64m["launch_sizes"],
                               "kernel_ms_total": sum(res64m["kern_ms"]),
                               "frac_fp64_mfma_12D2L2": 12.0 * D * D * L * L * props64 / kern64 / PEAK_FP64_MFMA,
                               "frac_fp64_mfma_8D2L2_executed":
                                   8.0 * D * D * L * L * props64 / kern64 / PEAK_FP64_MFMA,
                               "near_threshold_draws": res64m["near"]}
        if res64 is not None:
            out["batched_fp64"]["speedup_vs_plain_fp64"] = v64m / (res64["accepted"] / res64["wall"])
    if res16 is not None:
        props16 = C * sum(res16["launch_sizes"])
        kern16 = sum(res16["kern_ms"]) * 1e-3
        out["batched_bf16"] = {"value": res16["accepted"] / res16["wall"], "unit": UNIT,
                               "ms_per_step": res16["wall"] * 1e3 / args.steps,
                               "acceptance": res16["accepted"] / max(res16["proposed"], 1),
                               "tau_int_mean_energy": tau_int(res16["E"]),
                               "kernel": f"k_sampler_team<{-(-D // 16)},1,{res16['variant']}>",
                               "launch_steps": res16["launch_sizes"],
                               "kernel_ms_total": sum(res16["kern_ms"]),
                               "frac_bf16_mfma_12D2L2": 12.0 * D * D * L * L * props16 / kern16 / PEAK_BF16_MFMA,
                               "near_threshold_draws": res16["near"]}
    if not args.no_cpu:
        cb = run_cpu_oracle(inst)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        log(f"[bench] cpu oracle: {cb['value']:.2f} accepted/s on {cb['cores']} cores")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
