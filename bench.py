#!/usr/bin/env python3
"""Throughput of the checkerboard Metropolis sweep on one MI355X.

Default workload (the throughput configuration of the method, Sec. 2 /
Table 1 of the paper): 2D Ising model, L = 16384 (N = 2^28 spins), J = 1, hot
start from seed 2, beta = 0.4406868, 1000 sweeps with energy and
magnetisation measured every 10 sweeps.  One step = 10 sweeps + one
measurement written to a device ring (no host synchronisation inside the
timed region).  Ising spins are stored at one bit per site by default (the
same chain, bit for bit, as int8 spins); the int8 two-pass schedule, which is
HBM-bound, is measured beside it in the same run.  Other workloads
(--workload): 3D Ising L = 512, 2D XY L = 4096, 3D Heisenberg L = 256 (FP32
spins), the batched +-J spin glass (2048 lattices of L in {8,12,16,24,32},
32 temperatures), and the derivatives of ln Z (256 chains of a 2D L = 64
lattice with Gaussian couplings: sampling sweeps, then the covariance replay).

Prints one JSON line:
  value     spin-flip attempts per ns over the whole timed region;
  roofline  the dominant kernel's average launch time (step time over kernel
            launches, HIP events on the kernel's stream inside the timed
            region) against its bound: HBM (algorithmic bytes per launch over
            8 TB/s) or, for the bit-packed and tiled kernels, the VALU (issued
            32-bit lane operations from the committed rocprofv3 instruction
            count over 78.6 Tops/s); `traffic` is the HBM bytes per launch read
            from the committed rocprofv3 counter summary when it was taken on
            the current kernel sources, else null;
  int8_two_pass  the same workload with int8 spins (its HBM roofline);
  cpu_baseline  the FP64 CPU oracle timed on the host on a bounded sample of
            the same workload, whose result is also compared with the GPU's.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0
# VALU peak in 32-bit lane operations per second: the FP32 vector rate of
# 157.3 TFLOP/s counts an FMA as two flops, i.e. 78.6e12 lane operations/s
# (256 CUs x 2.4 GHz x 128 lanes: two VALU instructions per SIMD quad-cycle)
VALU_PEAK_TOPS = 78.6
# One VALU instruction per SIMD per quad-cycle (a wave64 instruction over the
# 16-lane SIMD): 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 lane
# operations/s, the issue ceiling of code whose instructions do not pair
VALU_ISSUE_PEAK_TOPS = 39.3

# Proposal widths giving 50 +- 5 % acceptance at the benchmark temperatures
# (found with the oracle on small lattices; checked by a CPU test).
XY_DELTA = 1.63        # rotation angle uniform in [-delta, delta]
HEIS_DELTA = 2.058     # half-angle of the spherical cap

WORKLOADS = {
    "ising2d": dict(d=2, n=1, L=16384, seed=2, beta=0.4406868),
    "ising3d": dict(d=3, n=1, L=512, seed=3, beta=0.2216546),
    "xy": dict(d=2, n=2, L=4096, seed=5, beta=1.12, delta=XY_DELTA, renorm=100),
    "heisenberg": dict(d=3, n=3, L=256, seed=6, beta=0.693, delta=HEIS_DELTA, renorm=100),
    "batched": dict(d=3, n=1, lattices=2048, Ls=(8, 12, 16, 24, 32), seed=4, betas=32,
                    beta_lo=0.5, beta_hi=3.0),
    "chains": dict(d=2, n=1, L=64, chains=256, seed=8, beta=0.4, J_mean=1.0, J_sigma=0.1),
}

# Source files of each dominant kernel (a counter summary is valid only for
# the sources it was taken on).
KERNEL_SOURCES = {
    "ising_stream": ["ising.hip", "chunk.hpp", "device.hpp", "launch_args.hpp", "reduce.hpp"],
    "ising_fused": ["fused.hip", "chunk.hpp", "device.hpp", "launch_args.hpp", "reduce.hpp"],
    "ising_packed": ["packed.hip", "packed.hpp", "chunk.hpp", "device.hpp", "launch_args.hpp",
                     "reduce.hpp"],
    "ising_tiles": ["tiles.hip", "packed.hpp", "chunk.hpp", "device.hpp", "launch_args.hpp"],
    "ising_tiles_packed": ["tiles.hip", "packed.hpp", "chunk.hpp", "device.hpp", "launch_args.hpp"],
    "xy_stream": ["continuous.hip", "chunk.hpp", "device.hpp", "launch_args.hpp"],
    "heisenberg_stream": ["continuous.hip", "chunk.hpp", "device.hpp", "launch_args.hpp"],
    "batch": ["batch.hip", "packed.hpp", "chunk.hpp", "device.hpp", "launch_args.hpp", "reduce.hpp"],
    "chains": ["chains.hip", "chunk.hpp", "device.hpp", "launch_args.hpp"],
    "probe": ["probe.hip", "device.hpp"],
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="ising2d")
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps of 10 sweeps + 1 measurement (default: 100, i.e. 1000 "
                         "sweeps; batched and chains: 1 step of 10^4 sweeps)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--sweeps-per-step", type=int, default=None,
                    help="sweeps per timed step (default 10; batched: 10000 in one launch)")
    ap.add_argument("--measure-every", type=int, default=10,
                    help="batched: E/M of every lattice every this many sweeps, inside the launch")
    ap.add_argument("--schedule", choices=["fused", "two-pass"], default="two-pass",
                    help="2D Ising only -- fused: one kernel per sweep with ping-pong buffers "
                         "(2 B/attempt); two-pass: one in-place kernel per colour (3 B/attempt)")
    ap.add_argument("--spins", choices=["packed", "int8"], default="packed",
                    help="Ising plain sweeps: one bit per site (default; the int8 two-pass "
                         "line is measured beside it) or int8 -- the same chain")
    ap.add_argument("--no-int8-line", action="store_true",
                    help="skip the int8 two-pass comparison line of a packed run")
    ap.add_argument("--tile", type=int, default=0,
                    help="Ising workloads: the tiled k-hit schedule with tiles of this edge")
    ap.add_argument("--hits", type=int, default=100, help="k of the tiled schedule")
    ap.add_argument("--heatbath", action="store_true", help="Ising workloads: heat-bath rule")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate host time of the oracle baseline (0 = skip)")
    ap.add_argument("--no-batched", action="store_true",
                    help="default 2D line: skip the batched spin-glass comparison attached to it")
    ap.add_argument("--no-extra", action="store_true",
                    help="default 2D line: skip the 3D Ising, XY, Heisenberg and chains objects "
                         "attached to it")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default band heights (the default run times every band "
                         "height of the lattice's kernel first and keeps the fastest)")
    ap.add_argument("--probes", action="store_true",
                    help="measure the ceilings instead of a workload: device copies of 32 MiB, "
                         "256 MiB and 1 GiB, Philox4x32-10 blocks alone, and the integer VALU "
                         "issue rate (probe kernels of the library)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one 1 GiB device copy before the timed region (calibrates the "
                         "HBM byte counters of a profiler run)")
    return ap.parse_args()


def sources_digest(kernel):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(kernel, []):
        with open(os.path.join(ROOT, "paper_1107_5463_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current sources of the kernel."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("sources_sha256_16") != sources_digest(kernel):
        return None
    return rec.get("hbm_bytes_per_launch")


def measured_probe(name):
    """A ceiling measured on the box by a committed probe (profiles/probe_*.json)."""
    path = os.path.join(ROOT, "profiles", f"probe_{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        return json.load(fh).get("value")


def host_cpu():
    """CPU model and processor count of the host the oracle ran on."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count()}


def copy_probe(torch, device):
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device=device).fill_(1)
    b = torch.empty(n, dtype=torch.uint8, device=device)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def copy_ceiling(torch, device, nbytes):
    """Device-to-device copy rate (read + write GB/s) of an nbytes buffer, the
    best of 10 copies timed with HIP events: a ceiling for streaming kernels
    of that footprint."""
    a = torch.empty(nbytes, dtype=torch.uint8, device=device).fill_(1)
    b = torch.empty(nbytes, dtype=torch.uint8, device=device)
    b.copy_(a)
    torch.cuda.synchronize()
    best = None
    for _ in range(10):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    return round(2 * nbytes / (best * 1e-3) / 1e9, 1)


def oracle_rate(fn, attempts_per_call, budget_s):
    """Calls fn until budget_s has passed (at least once); attempts/ns."""
    t0 = time.perf_counter()
    calls = 0
    while True:
        fn()
        calls += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            return calls * attempts_per_call / (el * 1e9), calls, el


def timed_steps(lat, beta, K, W, S, torch):
    """W untimed steps, then K timed steps of S sweeps + one measurement into
    a device ring; HIP events on the lattice's stream.  Returns (ms, wall s,
    last observables)."""
    st = lat.stream
    ring = torch.zeros((max(K, 1), 8), dtype=torch.int64, device=lat.device)
    for _ in range(W):
        lat.sweep_measure(beta, S, ring[0])
    torch.cuda.synchronize()
    ev_start = torch.cuda.Event(enable_timing=True)
    ev_end = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev_start.record(st)
    for k in range(K):
        lat.sweep_measure(beta, S, ring[k])
    ev_end.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    obs = lat.decode_obs(ring[K - 1:K])[0] if K else None
    return ev_start.elapsed_time(ev_end), wall, obs


def kernel_model(kname, n, N, sweeps, tile, hits):
    """(launches, algorithmic HBM bytes per launch, schedule) of the dominant kernel."""
    if kname in ("ising_tiles", "ising_tiles_packed"):
        # one launch per tile colour: its half of both planes read and written once
        return 2 * sweeps, 1.0 * N, f"tiled k-hit, T={tile}, k={hits}"
    if kname == "ising_packed":
        return 2 * sweeps, 1.5 * N / 8, "two-pass colour-split, in place, one bit per site"
    if kname == "ising_fused":
        return sweeps, 2.0 * N, "fused one-pass, ping-pong buffers"
    if n == 1:
        return 2 * sweeps, 1.5 * N, "two-pass colour-split, in place"
    # own colour read + written and other colour read, n FP32 components
    return 2 * sweeps, 1.5 * N * n * 4, "two-pass colour-split, in place, FP32 components"


def hbm_roofline(kname, workload, bytes_per_launch, kernel_ms):
    achieved = bytes_per_launch / (kernel_ms * 1e-3) / 1e9
    return {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": measured_traffic(kname, workload),
        "kernel": kname,
        "kernel_avg_us": round(kernel_ms * 1e3, 3),
        "algorithmic_bytes_per_launch": int(bytes_per_launch),
    }


def valu_roofline(kname, workload, kernel_ms, bytes_per_launch, attempts_per_launch,
                  variant=None):
    """VALU-bound kernels: issued 32-bit lane operations per second from the
    committed VALU instruction count per launch (rocprofv3 SQ_INSTS_VALU x 64
    lanes), valid only for the kernel sources and the variant (schedule, rule)
    it was taken on.  A count taken on launches of another length (sweeps per
    launch) is scaled by the attempts per launch; `counted_attempts_per_launch`
    then differs from `attempts_per_launch`."""
    rec = None
    path = os.path.join(ROOT, "profiles", f"{kname}_{workload}_valu.json")
    if os.path.exists(path):
        with open(path) as fh:
            recs = json.load(fh)
        # one record, or a list of records of different variants
        for r in recs if isinstance(recs, list) else [recs]:
            if r.get("sources_sha256_16") == sources_digest(kname) and r.get("variant") == variant:
                rec = r
    achieved = None
    if rec is not None:
        lane_ops = rec["valu_lane_ops_per_launch"] * attempts_per_launch / rec["attempts_per_launch"]
        achieved = lane_ops / (kernel_ms * 1e-3) / 1e12
    probe = measured_probe("valu_issue")
    return {
        "bound": "alu",
        "achieved": None if achieved is None else round(achieved, 2),
        "peak": VALU_PEAK_TOPS,
        "unit": "Tops/s",
        "frac": None if achieved is None else round(achieved / VALU_PEAK_TOPS, 4),
        "issue_peak": VALU_ISSUE_PEAK_TOPS,
        "frac_issue": None if achieved is None else round(achieved / VALU_ISSUE_PEAK_TOPS, 4),
        "probe_ceiling": probe,
        "frac_probe": None if (achieved is None or not probe) else round(achieved / probe, 4),
        "lane_ops_per_attempt": None if rec is None else rec.get("lane_ops_per_attempt"),
        "attempts_per_launch": int(attempts_per_launch),
        "counted_attempts_per_launch": None if rec is None else rec["attempts_per_launch"],
        "traffic": measured_traffic(kname, workload),
        "kernel": kname,
        "kernel_avg_us": round(kernel_ms * 1e3, 3),
        "algorithmic_bytes_per_launch": int(bytes_per_launch),
        "hbm_frac": round(bytes_per_launch / (kernel_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
    }


def run_lattice(args, wl, torch, smc):
    d, n, L = wl["d"], wl["n"], wl["L"]
    N = L ** d
    special = bool(args.tile or args.heatbath or args.schedule == "fused")
    packed = n == 1 and args.spins == "packed" and not special
    fused = args.schedule == "fused" and n == 1 and not (args.tile or args.heatbath)
    if n > 1:
        kw = dict(delta=wl["delta"], renorm_every=wl["renorm"])
    else:
        kw = dict(packed=packed, heatbath=args.heatbath, tile=args.tile,
                  hits=args.hits if args.tile else 0)
    lat = smc.Lattice(d, n, L, seed=wl["seed"], fused=fused, **kw)
    default_rows = lat.kernel()[1]
    if not args.no_autotune:
        lat.autotune(wl["beta"])
    if args.copy_probe:
        copy_probe(torch, lat.device)
    K = args.steps if args.steps is not None else 100
    W = args.warmup
    S = args.sweeps_per_step if args.sweeps_per_step is not None else 10
    beta = wl["beta"]
    total_ms, wall, obs = timed_steps(lat, beta, K, W, S, torch)
    sweeps = K * S
    hits = args.hits if (n == 1 and args.tile) else 1
    attempts = N * sweeps * hits
    kname, band_rows = lat.kernel()
    launches, bytes_per_launch, schedule = kernel_model(kname, n, N, sweeps, args.tile, args.hits)
    # the step time also holds the measurement finish (and renormalisation)
    # kernels: a conservative average of the dominant kernel
    kernel_ms = total_ms / launches
    if kname in ("ising_packed", "ising_tiles", "ising_tiles_packed"):
        variant = None
        if kname in ("ising_tiles", "ising_tiles_packed"):
            variant = f"T={args.tile} k={args.hits} {'heat bath' if args.heatbath else 'Metropolis'}"
        roof = valu_roofline(kname, args.workload, kernel_ms, bytes_per_launch,
                             attempts / launches, variant)
    else:
        roof = hbm_roofline(kname, args.workload, bytes_per_launch, kernel_ms)
    what = {1: "Ising", 2: "XY", 3: "Heisenberg"}[n]
    result = {
        "metric": "spin-flip attempts/ns + %HBM peak, 2D Ising L=16384; batched vs plain",
        "value": round(attempts / (total_ms * 1e6), 2),
        "unit": "attempts/ns",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(total_ms / max(K, 1), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("u1" if packed else "i8") if n == 1 else "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{d}D {what} L={L} (N={N}), J=1, beta={beta}, "
                        + ("spins at one bit per site, " if packed else "")
                        + ("heat bath, " if args.heatbath and n == 1 else "")
                        + (f"tiles T={args.tile} k={args.hits} ({hits} attempts per site "
                           "per sweep), " if args.tile and n == 1 else "")
                        + f"{'hot' if n == 1 else 'random'} start seed {wl['seed']}, {sweeps} "
                        f"checkerboard sweeps, E/M every {S} sweeps"
                        + (f", delta={wl['delta']}, renormalise every {wl['renorm']}" if n > 1 else ""),
            "d": d, "n": n, "L": L, "sweeps": sweeps, "measure_every": S,
            "schedule": schedule, "kernel": kname, "rows_per_band": band_rows,
            "rows_autotuned": not args.no_autotune, "rows_default": default_rows,
        },
        "roofline": roof,
        "pct_hbm_peak": round(100 * bytes_per_launch / (kernel_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 2),
        "wall_s": round(wall, 3),
        "final_obs": None if obs is None else {"E": obs.E, "M": list(obs.M[:n]), "sweep": obs.sweep},
    }
    if roof["bound"] == "hbm":
        # a plain device copy of the spin buffer's footprint, for context
        # next to the 8 TB/s peak
        roof["copy_ceiling_GBps"] = copy_ceiling(torch, lat.device,
                                                 lat.spins.numel() * lat.spins.element_size())
    if packed and not args.no_int8_line:
        # the same chain with int8 spins: the HBM-bound two-pass schedule
        lat8 = smc.Lattice(d, n, L, seed=wl["seed"])
        if not args.no_autotune:
            lat8.autotune(beta)
        ms8, _, obs8 = timed_steps(lat8, beta, K, W, S, torch)
        k8, rows8 = lat8.kernel()
        l8, b8, sch8 = kernel_model(k8, n, N, sweeps, 0, 1)
        roof8 = hbm_roofline(k8, args.workload, b8, ms8 / l8)
        roof8["copy_ceiling_GBps"] = copy_ceiling(torch, lat8.device,
                                                  lat8.spins.numel() * lat8.spins.element_size())
        result["int8_two_pass"] = {
            "value": round(attempts / (ms8 * 1e6), 2),
            "unit": "attempts/ns",
            "ms_per_step": round(ms8 / max(K, 1), 4),
            "schedule": sch8, "rows_per_band": rows8,
            "roofline": roof8,
            "same_final_state": bool(obs8 is not None and obs is not None and obs8.E_int == obs.E_int
                                     and obs8.M_int == obs.M_int),
        }
        del lat8

    if args.cpu_seconds > 0:
        sys.path.insert(0, ROOT)
        import oracle

        kwo = {} if n == 1 else dict(delta=wl["delta"], renorm_every=wl["renorm"])
        ref = oracle.OracleLattice(d, n, L, wl["seed"], **kwo)
        if n == 1 and (args.tile or args.heatbath):
            rule = "heatbath" if args.heatbath else "metropolis"
            one = lambda: ref.sweep_rule(beta, 1, rule, args.tile, args.hits if args.tile else 1)
        else:
            one = lambda: ref.sweep(beta, 1)
        rate, calls, el = oracle_rate(one, N * hits, args.cpu_seconds)
        gpu = smc.Lattice(d, n, L, seed=wl["seed"], **kw)
        gpu.sweep(beta, calls)
        go, ro = gpu.measure(), ref.measure()
        if n == 1:
            parity = bool(go.E_int == ro.E_int and go.M_int == ro.M_int)
            pname = "parity_E_M_after_sample"
        else:
            # FP32 chains leave the FP64 one after a few sweeps (near-threshold
            # decisions); report the relative energy difference instead
            parity = round(abs(go.E - ro.E) / max(1.0, abs(ro.E)), 6)
            pname = "rel_E_diff_after_sample"
        cores = oracle.num_threads()
        # the same oracle on one core (at least one sweep, about a third of
        # the time budget), then all cores again
        oracle.set_num_threads(1)
        ref1 = oracle.OracleLattice(d, n, L, wl["seed"], **kwo)
        if n == 1 and (args.tile or args.heatbath):
            one1 = lambda: ref1.sweep_rule(beta, 1, rule, args.tile, args.hits if args.tile else 1)
        else:
            one1 = lambda: ref1.sweep(beta, 1)
        rate1, calls1, el1 = oracle_rate(one1, N * hits, args.cpu_seconds / 3)
        oracle.set_num_threads(cores)
        result["cpu_baseline"] = {
            "value": round(rate, 4),
            "unit": "attempts/ns",
            "cores": cores,
            "kind": "oracle",
            "sample": f"first {calls} sweeps of the same {d}D L={L} lattice from the same start "
                      f"({N * calls * hits} attempts, {el:.1f} s)",
            pname: parity,
            "single_core": {"value": round(rate1, 4), "unit": "attempts/ns", "cores": 1,
                            "sample": f"first {calls1} sweeps ({el1:.1f} s)"},
            "host": host_cpu(),
        }
    return result


def run_batched(args, wl, torch, smc):
    d, nl = wl["d"], wl["lattices"]
    Ls = [wl["Ls"][r % len(wl["Ls"])] for r in range(nl)]
    betas = [wl["beta_lo"] + (wl["beta_hi"] - wl["beta_lo"]) * (r % wl["betas"]) / (wl["betas"] - 1)
             for r in range(nl)]
    sites = sum(L ** d for L in Ls)
    b = smc.Batch(d, Ls, betas, seed=wl["seed"], J_kind=smc.J_PM)
    threads, largest_first = b.autotune()
    b.use_graph(True)
    st = b.stream
    # one step = one persistent launch of S sweeps recording E and M of every
    # lattice every `every` sweeps
    K = args.steps if args.steps is not None else 1
    W = args.warmup
    S = args.sweeps_per_step if args.sweeps_per_step is not None else 10000
    every = args.measure_every
    if every < 1 or S % every:
        sys.exit("--measure-every must divide --sweeps-per-step")
    obs = torch.zeros((S // every, nl, 8), dtype=torch.int64, device=b.device)
    for _ in range(W):
        b.sweep(S, obs, every=every)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(st)
    for _ in range(K):
        b.sweep(S, obs, every=every)
    ev1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = ev0.elapsed_time(ev1)
    sweeps = K * S
    value = sites * sweeps / (total_ms * 1e6)

    # plain: the same kind of lattices one at a time through the single-lattice path
    plain_lats = [smc.Lattice(d, 1, Ls[r], seed=wl["seed"], J_kind=smc.J_PM, replica=r)
                  for r in range(2 * len(wl["Ls"]))]
    ps = 20
    for lt, r in zip(plain_lats, range(len(plain_lats))):
        lt.sweep(betas[r], 2)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(plain_lats[0].stream)
    for lt, r in zip(plain_lats, range(len(plain_lats))):
        lt.sweep(betas[r], ps)
    e1.record(plain_lats[0].stream)
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1)
    plain_value = sum(lt.N for lt in plain_lats) * ps / (plain_ms * 1e6)

    # spins + couplings cross HBM once per call (staged in LDS for all sweeps)
    cbytes = sum(L ** d for L in Ls) * (1 + d)
    result = {
        "metric": "spin-flip attempts/ns + %HBM peak, 2D Ising L=16384; batched vs plain",
        "value": round(value, 2),
        "unit": "attempts/ns",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(total_ms / max(K, 1), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8",
        "data": "synthetic",
        "config": {
            "workload": f"batched 3D +-J Edwards-Anderson: {nl} lattices, L in {list(wl['Ls'])} "
                        f"(lattice r has L[r % 5]), beta_r = 0.5 + 2.5 (r % 32) / 31, seed "
                        f"{wl['seed']}, {sweeps} sweeps in {K} persistent graph-replayed launch(es) of {S}, "
                        f"E/M of every lattice every {every} sweeps recorded inside the launch",
            "sites": sites, "sweeps": sweeps, "threads_per_lattice": threads,
            "largest_first": largest_first, "graph": True,
        },
        "plain": {"value": round(plain_value, 3), "unit": "attempts/ns",
                  "sample": f"{len(plain_lats)} of the lattices, one single-lattice sweep call "
                            f"each, {ps} sweeps"},
        "batched_vs_plain": round(value / plain_value, 1),
        # spins and couplings cross HBM once per launch (staged in LDS for all
        # sweeps): VALU-bound
        "roofline": valu_roofline("batch", "batched", total_ms / max(K, 1), 2 * cbytes,
                                  sites * S),
        "wall_s": round(wall, 3),
    }
    if args.cpu_seconds > 0:
        sys.path.insert(0, ROOT)
        import oracle

        done = []
        r = 0
        t0 = time.perf_counter()
        att = 0
        while time.perf_counter() - t0 < args.cpu_seconds and r < nl:
            ref = oracle.OracleLattice(d, 1, Ls[r], wl["seed"], J_kind=1, replica=r)
            ref.sweep(betas[r], 200)
            att += Ls[r] ** d * 200
            done.append(r)
            r += 1
        el = time.perf_counter() - t0
        result["cpu_baseline"] = {
            "value": round(att / (el * 1e9), 4),
            "unit": "attempts/ns",
            "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"lattices 0..{len(done) - 1} of the batch, 200 sweeps each ({att} attempts, "
                      f"{el:.1f} s)",
        }
    return result


def run_chains(args, wl, torch, smc):
    """Derivatives of ln Z: forward = sampling sweeps accumulating the bond
    products; backward = the covariance replay of the same sweeps."""
    import numpy as np
    d, L, nch = wl["d"], wl["L"], wl["chains"]
    N = L ** d
    rng = np.random.default_rng(wl["seed"])
    J_nat = rng.normal(wl["J_mean"], wl["J_sigma"], size=(d, N)).astype(np.float32)
    # natural -> colour-split layout of the couplings (site i = x + L y: colour
    # (x + y) & 1, in-colour index i >> 1)
    Js = np.empty((d, 2, N // 2), dtype=np.float32)
    i = np.arange(N)
    col = ((i % L) + (i // L)) & 1
    Js[:, col, i >> 1] = J_nat
    ch = smc.Chains(d, L, nch, wl["seed"], J=torch.from_numpy(Js).cuda())
    st = ch.stream
    # one step = one sampling call of S sweeps (default: the workload's 10^4
    # sweeps in one launch)
    K = args.steps if args.steps is not None else 1
    W = args.warmup
    S = args.sweeps_per_step if args.sweeps_per_step is not None else 10000
    beta = wl["beta"]
    for _ in range(W):
        ch.sample(beta, S)
    torch.cuda.synchronize()
    start = ch.spins.clone()
    t0 = ch.t
    acc = ch.bond_zeros()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record(st)
    for _ in range(K):
        ch.sample(beta, S, acc)
    ev[1].record(st)
    torch.cuda.synchronize()
    sweeps = K * S
    mean = ch.mean(acc, nch * sweeps)
    g = torch.randn(mean.shape, dtype=torch.float64, device=mean.device,
                    generator=torch.Generator(device=mean.device).manual_seed(1))
    gc = ch.dot(g, mean)
    cov_acc = torch.zeros_like(mean)
    G_acc = torch.zeros(2, dtype=torch.float64, device=mean.device)
    ch.spins.copy_(start)
    ch.t = t0
    torch.cuda.synchronize()
    ev[2].record(st)
    ch.covariance(beta, sweeps, g, gc, cov_acc, G_acc)
    ev[3].record(st)
    torch.cuda.synchronize()
    fwd_ms = ev[0].elapsed_time(ev[1])
    bwd_ms = ev[2].elapsed_time(ev[3])
    attempts = nch * N * sweeps
    result = {
        "metric": "spin-flip attempts/ns + %HBM peak, 2D Ising L=16384; batched vs plain",
        "value": round(attempts / (fwd_ms * 1e6), 2),
        "unit": "attempts/ns",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(fwd_ms / max(K, 1), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"derivatives of ln Z: {nch} chains of the 2D Ising L={L} lattice, J ~ "
                        f"N({wl['J_mean']}, {wl['J_sigma']}^2) (seed {wl['seed']}), beta={beta}, "
                        f"{sweeps} sweeps with the bond products summed after every sweep "
                        "(forward), then the covariance replay of the same sweeps (backward)",
            "chains": nch, "L": L, "sweeps": sweeps, "sweeps_per_launch": S,
            "kernel": ch.kernel(),
        },
        "backward": {"value": round(attempts / (bwd_ms * 1e6), 2), "unit": "attempts/ns",
                     "ms": round(bwd_ms, 3)},
        # each launch (S sweeps) reads and writes every chain's spins once and
        # stages the shared couplings from L2: VALU / LDS-bound
        "roofline": valu_roofline("chains", "chains", fwd_ms / max(K, 1), 2 * nch * N,
                                  nch * N * S),
    }
    if args.cpu_seconds > 0:
        sys.path.insert(0, ROOT)
        import oracle

        n_or = 8
        s0 = np.stack([oracle.init_ising(d, L, wl["seed"], replica=k) for k in range(n_or)])
        calls = [0]

        def one():
            oracle.chains_ising(d, L, wl["seed"], J_nat, beta, s0, 50)
            calls[0] += 1
        rate, c, el = oracle_rate(one, n_or * N * 50, args.cpu_seconds)
        result["cpu_baseline"] = {
            "value": round(rate, 4),
            "unit": "attempts/ns",
            "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{n_or} of the chains, 50 sweeps with bond sums, repeated {c} times "
                      f"({el:.1f} s)",
        }
    return result


PROBE_LANES = 1 << 20
PROBE_PHILOX_BLOCKS = 512
PROBE_VALU_ITERS = 4096


def run_probes(args, torch, smc):
    """Ceilings measured on this GPU: device copies (read + write GB/s, best of
    10), Philox blocks per ns with nothing else to do, and the issued VALU
    lane-operation rate of independent integer chains (instructions per lane
    and iteration from the committed counter record of the probe kernel)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    buf = torch.empty(PROBE_LANES, dtype=torch.int32, device=dev)
    st = torch.cuda.current_stream(dev)

    def best_ms(kind, reps):
        smc.probe(kind, PROBE_LANES, reps, buf)
        torch.cuda.synchronize()
        best = None
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            smc.probe(kind, PROBE_LANES, reps, buf)
            e1.record(st)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        return best

    ph_ms = best_ms("philox", PROBE_PHILOX_BLOCKS)
    va_ms = best_ms("valu", PROBE_VALU_ITERS)
    rec = None
    path = os.path.join(ROOT, "profiles", "probe_valu_counts.json")
    if os.path.exists(path):
        with open(path) as fh:
            r = json.load(fh)
        if r.get("sources_sha256_16") == sources_digest("probe"):
            rec = r
    out = {
        "metric": "ceilings measured by probes",
        "copy_GBps": {f"{mb}MiB": copy_ceiling(torch, dev, mb << 20) for mb in (32, 256, 1024)},
        "philox_blocks_per_ns": round(PROBE_LANES * PROBE_PHILOX_BLOCKS / (ph_ms * 1e6), 1),
        "philox_ms": round(ph_ms, 4),
        "valu_ms": round(va_ms, 4),
        "probe_lanes": PROBE_LANES,
    }
    if rec is not None:
        # issued VALU instructions (per lane) of one iteration or one block
        ops = rec["valu_per_lane_iteration"] * PROBE_LANES * PROBE_VALU_ITERS
        out["valu_issue_Tops"] = round(ops / (va_ms * 1e-3) / 1e12, 2)
        out["valu_per_philox_block"] = rec.get("valu_per_philox_block")
        if rec.get("valu_per_philox_block"):
            pops = rec["valu_per_philox_block"] * PROBE_LANES * PROBE_PHILOX_BLOCKS
            out["philox_Tops"] = round(pops / (ph_ms * 1e-3) / 1e12, 2)
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the multi-GPU (slab "
                                   "halo-exchange) path is not built", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import paper_1107_5463_amd as smc

    smc.load_library()
    if args.probes:
        print(json.dumps(run_probes(args, torch, smc)), flush=True)
        return
    wl = WORKLOADS[args.workload]
    if args.workload == "batched":
        result = run_batched(args, wl, torch, smc)
    elif args.workload == "chains":
        result = run_chains(args, wl, torch, smc)
    else:
        result = run_lattice(args, wl, torch, smc)
        special = bool(args.tile or args.heatbath or args.schedule == "fused")
        if args.workload == "ising2d" and not special and not args.no_batched:
            # the second half of the metric: the batched spin-glass workload
            # (one persistent launch of 10^4 sweeps) against the single-lattice path
            bargs = argparse.Namespace(**vars(args))
            bargs.steps, bargs.warmup, bargs.sweeps_per_step, bargs.cpu_seconds = 1, 1, None, 0
            bres = run_batched(bargs, WORKLOADS["batched"], torch, smc)
            result["batched"] = {k: bres[k] for k in ("value", "unit", "ms_per_step", "batched_vs_plain",
                                                      "plain", "roofline")}
            result["batched"]["workload"] = bres["config"]["workload"]
        if args.workload == "ising2d" and not special and not args.no_extra:
            attach_other_workloads(args, result, torch, smc)
    print(json.dumps(result), flush=True)


def attach_other_workloads(args, result, torch, smc):
    """The other throughput configurations, each with its own roofline, as
    objects of the default line (same GPU, same run; no CPU baseline): 3D
    Ising L = 512 (one bit per site, with its int8 two-pass line), 2D XY
    L = 4096 and 3D Heisenberg L = 256 (FP32 spins), the tiled k-hit schedule
    on the 2D lattice (T = 16 and 64, k = 100, Metropolis and heat bath) and
    on the 3D lattice (T = 16, k = 100), and the derivative chains (256
    chains of L = 64, forward and backward).  The batched
    spin-glass rate is set against the plain sweeps of the large lattices."""
    keep = ("value", "unit", "ms_per_step", "dtype", "roofline", "pct_hbm_peak")
    for name in ("ising3d", "xy", "heisenberg"):
        a = argparse.Namespace(**vars(args))
        a.workload, a.steps, a.sweeps_per_step, a.cpu_seconds = name, None, None, 0
        r = run_lattice(a, WORKLOADS[name], torch, smc)
        o = {k: r[k] for k in keep}
        o["workload"] = r["config"]["workload"]
        o["kernel"], o["rows_per_band"] = r["config"]["kernel"], r["config"]["rows_per_band"]
        o["rows_autotuned"] = r["config"]["rows_autotuned"]
        if "int8_two_pass" in r:
            o["int8_two_pass"] = r["int8_two_pass"]
        result[name] = o
        torch.cuda.empty_cache()
    # the paper's tiled k-hit schedule (k = 100) on the 2D lattice: its 16 x 16
    # tiles and tiles of 64, both at one bit per site in LDS, under the
    # Metropolis rule and the heat-bath rule
    for hb in (False, True):
        for T in (16, 64):
            a = argparse.Namespace(**vars(args))
            a.workload, a.cpu_seconds = "ising2d", 0
            a.tile, a.hits, a.heatbath = T, 100, hb
            a.steps, a.warmup, a.sweeps_per_step = 2, 1, 2
            r = run_lattice(a, WORKLOADS["ising2d"], torch, smc)
            o = {k: r[k] for k in ("value", "unit", "ms_per_step", "dtype", "roofline")}
            o["workload"] = r["config"]["workload"]
            o["kernel"] = r["config"]["kernel"]
            result[f"tiles{T}_heatbath" if hb else f"tiles{T}"] = o
            torch.cuda.empty_cache()
    # and the paper's 3D row: 3D L = 512, 16^3 tiles at one bit per site in LDS, k = 100
    a = argparse.Namespace(**vars(args))
    a.workload, a.cpu_seconds = "ising3d", 0
    a.tile, a.hits, a.heatbath = 16, 100, False
    a.steps, a.warmup, a.sweeps_per_step = 2, 1, 1
    r = run_lattice(a, WORKLOADS["ising3d"], torch, smc)
    o = {k: r[k] for k in ("value", "unit", "ms_per_step", "dtype", "roofline")}
    o["workload"] = r["config"]["workload"]
    o["kernel"] = r["config"]["kernel"]
    result["tiles16_3d"] = o
    torch.cuda.empty_cache()
    a = argparse.Namespace(**vars(args))
    a.workload, a.steps, a.sweeps_per_step, a.cpu_seconds = "chains", None, None, 0
    r = run_chains(a, WORKLOADS["chains"], torch, smc)
    result["chains"] = {k: r[k] for k in ("value", "unit", "ms_per_step", "dtype", "roofline",
                                          "backward")}
    result["chains"]["workload"] = r["config"]["workload"]
    result["chains"]["kernel"] = r["config"]["kernel"]
    b = result.get("batched")
    if b is not None:
        plain = {"ising2d_packed": result["value"],
                 "ising2d_int8": result.get("int8_two_pass", {}).get("value"),
                 "ising3d_packed": result["ising3d"]["value"],
                 "ising3d_int8": result["ising3d"].get("int8_two_pass", {}).get("value")}
        # per attempt: the batched launch against the plain sweep of one large
        # lattice (3D: the same lattice dimension as the batch)
        b["vs_plain_large"] = {k: (round(b["value"] / v, 3) if v else None)
                               for k, v in plain.items()}


if __name__ == "__main__":
    main()
