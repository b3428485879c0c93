"""Throughput of the differentiable MLS-MPM substep on one MI355X.

One step = one pass of the whole path over the workload: load the initial
state (device to device), forward S substeps with recording (checkpoints every
K, the particle sort at each checkpoint), then the backward from the
cotangent of L = sum_p x_p . w_p to the initial state and per-env parameters
(segments recomputed from checkpoints). Inputs are resident in HBM before the
timed region.

Default workload: 32 identical environments on 48^3 grids, 20,000 corotated
particles each (E = 1e4, nu = 0.25), 80 substeps at dt = 5e-5, checkpoint
interval 10. Metric: fwd+bwd particle-substeps/s of the batched mode; the
per-environment mode, forward-only rate and p50/p99 per-step latency are
reported beside it, with a roofline entry for the dominant kernel and the FP64
oracle timed on the host as the CPU baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# algorithmic bytes per particle per launch of each kernel class (FP32 state:
# x 12, v 12, C 36, F 36 = 96 B) -- grid-node traffic is counted separately
ALG_BYTES_PER_PARTICLE = {
    "p2g": 96,          # read x, v, C, F
    "g2p": 48 + 96,     # read x, F; write x, v, C, F
    "g2p_adj": 48 + 96 + 48,   # read x, F, the state cotangent; write the partial x/F cotangent
    "p2g_adj": 96 + 48 + 96,   # read state and partial cotangent; write the state cotangent
    "sort": 96 + 96 + 4 * 8,   # permute read + write, keys/values
    "g2p2g": 48 + 96,   # G2P's reads and writes; the next P2G takes the new state from registers
    # P2G adjoint k: read state k and the partial cotangent; G2P adjoint k - 1: read x, F of
    # state k - 1 (C of state k again, counted once) and write the partial cotangent
    "adj_pair": 96 + 48 + 48 + 48,
}
# algorithmic bytes per touched grid node per launch
ALG_BYTES_PER_NODE = {"p2g": 16, "g2p": 12, "grid": 16 + 12, "g2p_adj": 12 + 12, "p2g_adj": 16, "grid_adj": 16 + 12 + 16,
                      "g2p2g": 12 + 16, "adj_pair": 16 + 12 + 12}


# kernel symbol of each class for the library's default batched variants
KERNEL_SYMBOL = {"p2g": {0: "k_p2g_direct", 1: "k_p2g_lds", 2: "k_p2g_seg"},
                 "g2p": {0: "k_g2p_direct", 1: "k_g2p_lds"},
                 "g2p_adj": {0: "k_g2p_adjoint_direct", 1: "k_g2p_adjoint_lds", 2: "k_g2p_adjoint_seg"},
                 "p2g_adj": {0: "k_p2g_adjoint_direct", 1: "k_p2g_adjoint_lds"},
                 "g2p2g": {1: "k_g2p2g"}, "adj_pair": {1: "k_adj_pair"}}


def kernel_source_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("mpm_device.h", "mpm_kernels.h", "mpm_kernels.hip", "mpm_kernels_lds.hip"):
        with open(os.path.join(ROOT, "paper_2412_12089_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_instance(symbol: str, variant, tuned: dict, envs) -> str:
    """Name of the launched instantiation, as profilers print it: the LDS-staged
    kernels are templates over (persistent grid, LDS box nodes, material)."""
    if not variant:
        return symbol
    mats = sorted({e.material for e in envs})
    mat = mats[0] if tuned["SPECIALIZE"] and len(mats) == 1 else -1
    if symbol in ("k_g2p2g", "k_adj_pair"):   # no persistent-grid parameter
        return f"{symbol}<{384 if tuned['BOX'] else 1024}, {mat}>"
    n_items = sum(-(-e.n_particles // 256) for e in envs)
    persist = "true" if 0 < tuned["GRID_CAP"] < n_items else "false"
    mats = sorted({e.material for e in envs})
    mat = mats[0] if tuned["SPECIALIZE"] and len(mats) == 1 else -1
    return f"{symbol}<{persist}, {384 if tuned['BOX'] else 1024}, {mat}>"


def measured_traffic(workload: str, symbol: str):
    """HBM bytes per launch from the committed rocprofv3 counter runs, or None if
    there are none or the kernel sources changed since they were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha") != kernel_source_sha() or symbol not in rec.get("kernels", {}):
        return None
    return rec["kernels"][symbol]["bytes"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batched_corot",
                    choices=["batched_corot", "uneven_mixed", "dam_break", "single_nh", "handflip_shape"])
    ap.add_argument("--plain-steps", type=int, default=1, help="timed steps of the per-env mode (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-substeps", type=int, default=80, help="substeps per env of the oracle sample")
    ap.add_argument("--cpu-envs", type=int, default=2, help="envs of the oracle sample (about 10-20 s in all)")
    ap.add_argument("--profile", action="store_true", help="only run the batched steps (for rocprofv3)")
    ap.add_argument("--no-graphs", action="store_true", help="launch segments without hipGraph replay")
    ap.add_argument("--tune-ms", type=int, default=4000, help="autotuner budget (0: library defaults)")
    ap.add_argument("--set", default="", help="fixed library options instead of autotuning, e.g. P2G=2,G2P=0,BOX=1 "
                    "(a profiling run uses the choice an earlier timed run printed under 'autotuned')")
    ap.add_argument("--serve-seconds", type=float, default=5.0,
                    help="length of the Poisson request stream of the serving leg (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-slots", type=int, default=48)
    return ap.parse_args()


def touched_nodes(envs, wall_pad=2):
    """Grid nodes inside the stencils of the initial particles (per env, summed)."""
    total = 0
    for e in envs:
        b = np.floor(e.x.astype(np.float64) * e.n - 0.5).astype(np.int64)
        occ = np.zeros((e.n,) * 3, dtype=bool)
        for ox in range(3):
            for oy in range(3):
                for oz in range(3):
                    occ[b[:, 0] + ox, b[:, 1] + oy, b[:, 2] + oz] = True
        total += int(occ.sum())
    return total


def run_steps(batch, x0, w, S, steps, warmup, record=True, backward=True):
    import torch
    stream = batch.stream
    times = []
    for i in range(warmup + steps):
        if i == warmup:
            torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        batch.set_particles(*x0)
        batch.forward(S, record=record)
        if backward:
            batch.backward(gx=w)
        ev1.record(stream)
        if i >= warmup:
            times.append((ev0, ev1))
    torch.cuda.synchronize()
    batch.sync()
    ms = [a.elapsed_time(b) for a, b in times]
    return ms


def serving_leg(seconds, rate, slots, device):
    """Continuous batching of a seeded Poisson stream of single-env rollout requests."""
    import torch
    from paper_2412_12089_amd import scenes
    from paper_2412_12089_amd.server import GPUExecutor, Server
    reqs = scenes.serving_stream(seed=5, rate=rate, duration=seconds)
    ex = GPUExecutor(slots, n_cap=64, N_cap=100_000, chunk=10, device=device)
    free = torch.cuda.mem_get_info(device)[0]
    srv = Server(ex, budget_bytes=int(0.25 * free), chunk=10, keep_results=False)
    srv.run(reqs, realtime=True, timeout_s=max(120.0, 20 * seconds))
    st = srv.stats()
    ex.close()
    fwd = sum(r.env.n_particles * r.substeps for r in reqs)
    st.update({"rate_per_s": rate, "stream_s": seconds, "slots": slots, "budget_bytes": int(0.25 * free),
               "backward_fraction": sum(r.backward for r in reqs) / max(1, len(reqs)),
               "fwd_particle_substeps_demanded_per_s": fwd / seconds})
    return st


def cpu_baseline(wl, substeps, n_envs):
    """The FP64 oracle on a bounded sample: the first n_envs envs, `substeps` substeps each, forward + reverse."""
    import torch
    from oracle import mpm_oracle as O
    threads = torch.get_num_threads()
    done, t_all = 0, 0.0
    specs = wl.envs[:max(1, n_envs)]
    for i, spec in enumerate(specs):
        env, prm, st = O.env_from_spec(spec)
        cot = O.linear_loss_cotangent(wl.loss_weights[i], spec.n_particles)
        t0 = time.perf_counter()
        O.rollout_vjp(env, prm, st, substeps, cot)   # forward (stores states) + per-substep reverse
        t_all += time.perf_counter() - t0
        done += spec.n_particles * substeps
    return {"value": done / t_all, "unit": "particle-substeps/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(specs)} env(s) of {wl.name} ({done // substeps} particles), {substeps} substeps "
                      f"fwd+bwd each, {t_all:.1f} s wall"}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: environments never exchange data, so a multi-GPU run is "
              "independent single-GPU runs over disjoint env sets; run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2412_12089_amd import scenes
    from paper_2412_12089_amd.batch import Batch

    wl = scenes.WORKLOADS[args.workload]()
    S, K = wl.substeps, wl.ckpt_every
    envs = wl.envs
    N = sum(e.n_particles for e in envs)
    dev = torch.device("cuda:0")
    cat = lambda k: torch.from_numpy(np.concatenate([getattr(e, k) for e in envs], axis=0)).to(dev)
    x0 = (cat("x"), cat("v"), cat("C"), cat("F"))
    w = torch.from_numpy(np.concatenate(wl.loss_weights, axis=0)).to(dev)

    b = Batch(envs, max_substeps=S, ckpt_every=K, mode="batched", device=dev)
    from paper_2412_12089_amd import _capi
    if args.no_graphs:
        b.set_option(_capi.OPT_GRAPHS, 0)
    tune_s = None
    fixed = dict(kv.split("=") for kv in args.set.split(",") if kv)
    for k, v in fixed.items():
        b.set_option(getattr(_capi, "OPT_" + k.upper()), int(v))
    if args.tune_ms > 0 and not args.profile and not fixed:
        b.set_particles(*x0)
        t0 = time.perf_counter()
        b.autotune(args.tune_ms)
        tune_s = time.perf_counter() - t0
    tuned = {k: b.get_option(getattr(_capi, "OPT_" + k)) for k in ("P2G", "G2P", "G2P_ADJ", "P2G_ADJ", "MIN_RUN", "GRID_CAP", "MAX_RUN", "BOX", "SPECIALIZE", "FUSE", "FUSE_ADJ", "XCD")}
    ms = run_steps(b, x0, w, S, args.steps, args.warmup)
    if args.profile:
        # calibration for HBM byte counters: one plain 256 MiB device-to-device copy
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_ms_per_step": float(np.mean(ms)), "calibration_copy_bytes": 256 << 20}), flush=True)
        return
    step_ms = float(np.mean(ms))
    value = N * S / (step_ms * 1e-3)
    # forward-only rate
    fwd_ms = float(np.mean(run_steps(b, x0, w, S, max(1, args.steps // 2), 1, record=False, backward=False)))
    # roofline pass: per-kernel HIP events on the library's stream
    b.set_timing(True)
    b.set_particles(*x0)
    b.forward(S, record=True)
    classes = _capi.KERNEL_CLASSES
    kt_f = {k: b.kernel_time(k) for k in classes}
    b.backward(gx=w)
    kt_b = {k: b.kernel_time(k) for k in classes}   # includes the recomputed segments
    b.set_timing(False)
    kt = {}
    for k in classes:
        (mf, nf), (mb, nb) = kt_f[k], kt_b[k]
        n = nf + nb
        kt[k] = ((mf * nf + mb * nb) / n if n else 0.0, n)
    variant = {"p2g": b.get_option(_capi.OPT_P2G), "g2p": b.get_option(_capi.OPT_G2P),
               "g2p_adj": b.get_option(_capi.OPT_G2P_ADJ), "p2g_adj": b.get_option(_capi.OPT_P2G_ADJ),
               "g2p2g": b.get_option(_capi.OPT_FUSE), "adj_pair": b.get_option(_capi.OPT_FUSE_ADJ)}
    mem = b.memory_bytes()
    b.close()
    nodes = touched_nodes(envs)
    totals = {k: v[0] * v[1] for k, v in kt.items()}
    dom = max((k for k in totals if k in ALG_BYTES_PER_PARTICLE), key=lambda k: totals[k])
    dom_ms = kt[dom][0]
    alg_bytes = ALG_BYTES_PER_PARTICLE[dom] * N + ALG_BYTES_PER_NODE.get(dom, 0) * nodes
    achieved = alg_bytes / (dom_ms * 1e-3) / 1e9
    symbol = kernel_instance(KERNEL_SYMBOL.get(dom, {}).get(variant.get(dom), dom), variant.get(dom), tuned, envs)
    traffic = measured_traffic(wl.name, symbol)

    plain = None
    if args.plain_steps > 0:
        bp = Batch(envs, max_substeps=S, ckpt_every=K, mode="plain", device=dev)
        pms = run_steps(bp, x0, w, S, args.plain_steps, 1)
        bp.close()
        plain = N * S / (float(np.mean(pms)) * 1e-3)

    serving = None
    if args.serve_seconds > 0:
        serving = serving_leg(args.serve_seconds, args.serve_rate, args.serve_slots, dev)
    cpu = None if args.no_cpu_baseline else cpu_baseline(wl, args.cpu_substeps, args.cpu_envs)
    out = {
        "metric": "fwd+bwd particle-substeps/s (batched)",
        "value": value,
        "unit": "particle-substeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "envs": len(envs), "particles": N, "grid": envs[0].n,
                   "substeps": S, "ckpt_every": K, "material": scenes.MATERIAL_NAMES[envs[0].material]},
        "autotuned": tuned,
        "autotune_s": tune_s,
        "per_env_value": plain,
        "batched_over_per_env": (value / plain) if plain else None,
        "fwd_only_value": N * S / (fwd_ms * 1e-3),
        "p50_ms": float(np.percentile(ms, 50)),
        "p99_ms": float(np.percentile(ms, 99)),
        "hbm_resident_bytes": mem,
        "kernel_ms": {k: v[0] for k, v in kt.items()},
        "kernel_launches_per_step": {k: v[1] for k, v in kt.items()},
        "roofline": {"bound": "hbm", "kernel": symbol, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "alg_bytes_per_launch": alg_bytes, "touched_nodes": nodes, "kernel_ms": dom_ms},
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
