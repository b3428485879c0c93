"""Throughput of the differentiable MLS-MPM substep on one MI355X.

One step = one pass of the whole path over the workload: load the initial
state (device to device), forward S substeps with recording (checkpoints every
K, the particle sort at each checkpoint), then the backward from the
cotangent of L = sum_p x_p . w_p to the initial state and per-env parameters
(segments recomputed from checkpoints). Inputs are resident in HBM before the
timed region.

Headline workload: the large fluid scene -- 16 environments on 96^3 grids,
200,000 weakly compressible (Tait) particles each in a dam-break column held
by a kinematic gate withdrawn at 0.2 m/s, 100 substeps at dt = 2e-5,
checkpoint interval 20. Metric: fwd+bwd particle-substeps/s of the batched
mode. Reported beside it: the per-environment mode, the forward-only rate,
p50/p99 per-step latency, the batched corotated (32 x 20,000) and uneven mixed
(64 envs, 5k-60k) workloads, the continuous-batching server on a Poisson
stream (p50/p99 latency and aggregate particle-substeps/s), a roofline entry
for the dominant kernel, and the FP64 oracle timed on the host as the CPU
baseline.
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

# Algorithmic bytes each kernel must move, per particle and per touched grid
# node of one launch. FP32 state: x 12, v 12, C 36, F 36 = 96 B per particle.
# A forward substep reads and writes the state once (192 B per particle) and
# moves 28 B per touched node (m, P 16 B; v 12 B); the adjoint of a substep
# reads the state and the incoming cotangent and writes the outgoing one
# (288 B per particle) and moves twice the forward's grid bytes (56 B per node).
# A kernel that carries out a whole substep (the fused ones) is charged those
# figures; a kernel that carries out part of one is charged what that part
# reads and writes.
ALG_BYTES_PER_PARTICLE = {
    "p2g": 96,                # read x, v, C, F
    "g2p": 48 + 96,           # read x, F; write x, v, C, F
    "g2p_adj": 48 + 96 + 48,  # read x, F, the state cotangent; write the partial (x, F) cotangent
    "p2g_adj": 96 + 48 + 96,  # read the state and the partial cotangent; write the state cotangent
    "sort": 96 + 96 + 4 * 8,  # permute read + write, keys/values
    "g2p2g": 192,             # one forward substep (G2P of k + P2G of k + 1)
    "adj_pair": 288,          # one adjoint substep (P2G adjoint of k + G2P adjoint of k - 1)
}
ALG_BYTES_PER_NODE = {"p2g": 16, "g2p": 12, "grid": 16 + 12, "g2p_adj": 12 + 12, "p2g_adj": 16,
                      "grid_adj": 16 + 12 + 16, "g2p2g": 28, "adj_pair": 56}

# kernel symbol of each class for the library's batched variants
KERNEL_SYMBOL = {"p2g": {0: "k_p2g_direct", 1: "k_p2g_lds", 2: "k_p2g_seg", 3: "k_p2g_pull"},
                 "g2p": {0: "k_g2p_direct", 1: "k_g2p_lds"},
                 "g2p_adj": {0: "k_g2p_adjoint_direct", 1: "k_g2p_adjoint_lds", 2: "k_g2p_adjoint_seg",
                             3: "k_g2p_adjoint_pull"},
                 "p2g_adj": {0: "k_p2g_adjoint_direct", 1: "k_p2g_adjoint_lds"},
                 "g2p2g": {1: "k_g2p2g", 2: "k_g2p2g_pull"}, "adj_pair": {1: "k_adj_pair"}}
OPTION_NAMES = ("P2G", "G2P", "G2P_ADJ", "P2G_ADJ", "MIN_RUN", "GRID_CAP", "MAX_RUN", "BOX", "SPECIALIZE", "FUSE",
                "FUSE_ADJ", "XCD", "GRID_LIST")


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
    if symbol == "k_g2p2g_pull":   # no persistent-grid parameter, the pull box budgets
        return f"{symbol}<{1024 if tuned['BOX'] else 2048}, {mat}>"
    if symbol in ("k_g2p2g", "k_adj_pair"):   # no persistent-grid parameter
        return f"{symbol}<{384 if tuned['BOX'] else 1024}, {mat}>"
    n_items = sum(-(-e.n_particles // 256) for e in envs)
    persist = "true" if 0 < tuned["GRID_CAP"] < n_items else "false"
    if symbol.endswith("_pull"):   # the pull scatters' larger box budgets
        return f"{symbol}<{persist}, {1024 if tuned['BOX'] else 2048}, {mat}>"
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


def progress(msg):
    """A progress line on stderr (the JSON result is the one line on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="dam_break",
                    choices=["batched_corot", "uneven_mixed", "dam_break", "single_nh", "handflip_shape",
                             "handflip_gripper"])
    ap.add_argument("--extra", default="batched_corot,uneven_mixed",
                    help="further workloads timed (autotuned, batched, fwd+bwd) and reported beside the headline")
    ap.add_argument("--plain-steps", type=int, default=1, help="timed steps of the per-env mode (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-substeps", type=int, default=5, help="substeps of each oracle run (fwd+bwd)")
    ap.add_argument("--cpu-envs", type=int, default=1, help="envs of the oracle sample")
    ap.add_argument("--cpu-runs", type=int, default=3, help="oracle runs; the median rate is reported")
    ap.add_argument("--profile", action="store_true", help="only run the batched steps (for rocprofv3)")
    ap.add_argument("--no-graphs", action="store_true", help="launch segments without hipGraph replay")
    ap.add_argument("--tune-ms", type=int, default=4000, help="autotuner budget (0: library defaults)")
    ap.add_argument("--set", default="", help="fixed library options instead of autotuning, e.g. P2G=3,G2P=0,BOX=1 "
                    "(a profiling run uses the choice an earlier timed run printed under 'autotuned')")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the Poisson request stream of the serving leg (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-slots", type=int, default=48)
    ap.add_argument("--fem-envs", type=int, default=4096, help="jumper envs of the FEM leg (0: skip)")
    ap.add_argument("--fem-frames", type=int, default=5, help="timed 80-substep frames of the FEM leg")
    ap.add_argument("--fem-only", action="store_true", help="run only the FEM leg and print its JSON (profiling)")
    ap.add_argument("--rb-envs", type=int, default=65536, help="hand envs of the rigid-body leg (0: skip)")
    ap.add_argument("--rb-frames", type=int, default=10, help="timed 16-substep frames of the rigid-body leg")
    ap.add_argument("--rb-only", action="store_true", help="run only the rigid-body leg and print its JSON")
    return ap.parse_args()


def touched_nodes(envs):
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
    """Per-step durations (ms) from HIP events recorded on the library's stream."""
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
    return [a.elapsed_time(b) for a, b in times]


def inputs(wl, dev):
    import torch
    cat = lambda k: torch.from_numpy(np.concatenate([getattr(e, k) for e in wl.envs], axis=0)).to(dev)
    x0 = (cat("x"), cat("v"), cat("C"), cat("F"))
    w = torch.from_numpy(np.concatenate(wl.loss_weights, axis=0)).to(dev)
    return x0, w


def tuned_batch(wl, dev, args, fixed=None):
    """A batched-mode batch with the autotuner's (or the fixed) options."""
    from paper_2412_12089_amd import _capi
    from paper_2412_12089_amd.batch import Batch
    b = Batch(wl.envs, max_substeps=wl.substeps, ckpt_every=wl.ckpt_every, mode="batched", device=dev)
    if args.no_graphs:
        b.set_option(_capi.OPT_GRAPHS, 0)
    for k, v in (fixed or {}).items():
        b.set_option(getattr(_capi, "OPT_" + k.upper()), int(v))
    tune_s = None
    if args.tune_ms > 0 and not args.profile and not fixed:
        x0, _ = inputs(wl, dev)
        b.set_particles(*x0)
        t0 = time.perf_counter()
        b.autotune(args.tune_ms)
        tune_s = time.perf_counter() - t0
    tuned = {k: b.get_option(getattr(_capi, "OPT_" + k)) for k in OPTION_NAMES}
    return b, tuned, tune_s


def extra_workload(name, dev, args):
    """Batched fwd+bwd rate of another workload (autotuned), in the same units."""
    from paper_2412_12089_amd import scenes
    wl = scenes.WORKLOADS[name]()
    N = sum(e.n_particles for e in wl.envs)
    b, tuned, _ = tuned_batch(wl, dev, args)
    x0, w = inputs(wl, dev)
    ms = run_steps(b, x0, w, wl.substeps, max(3, args.steps), 1)
    b.close()
    step = float(np.median(ms))
    return {"value": N * wl.substeps / (step * 1e-3), "unit": "particle-substeps/s", "ms_per_step": step,
            "envs": len(wl.envs), "particles": N, "substeps": wl.substeps, "ckpt_every": wl.ckpt_every,
            "autotuned": tuned}


def serving_leg(seconds, rate, slots, device):
    """Continuous batching (the library's server) of a seeded Poisson stream of single-env rollout requests."""
    import torch
    from paper_2412_12089_amd import scenes
    from paper_2412_12089_amd.server import Server
    reqs = scenes.serving_stream(seed=5, rate=rate, duration=seconds)
    free = torch.cuda.mem_get_info(device)[0]
    budget = int(0.25 * free)
    srv = Server(slots, n_cap=64, N_cap=100_000, chunk=10, budget_bytes=budget, device=device, keep_results=False)
    srv.run(reqs, realtime=True, timeout_s=max(120.0, 20 * seconds))
    st = srv.stats()
    srv.close()
    fwd = sum(r.env.n_particles * r.substeps for r in reqs)
    st.update({"rate_per_s": rate, "stream_s": seconds, "slots": slots, "budget_bytes": budget,
               "backward_fraction": sum(r.backward for r in reqs) / max(1, len(reqs)),
               "particle_substeps_demanded_per_s": fwd / seconds})
    return st


def fem_leg(n_envs, frames, dev):
    """The tetrahedral FEM path on jumper-shaped soft bodies (199 nodes, 480
    elements each): per 80-substep frame a recorded forward and its adjoint
    (cotangents of the initial state, the activations and the parameters),
    timed with HIP events on the library's stream."""
    import torch
    from paper_2412_12089_amd import fem_scenes as FS
    from paper_2412_12089_amd.fem import FemBatch
    w = FS.soft_jumper(seed=7, n_envs=n_envs, substeps=80)
    E, n, T, S = w.n_envs, w.X.shape[1], w.tets.shape[0], w.substeps
    b = FemBatch(w.tets, E, n, S, w.dt, w.gravity, dev)
    b.set_rest(torch.from_numpy(w.X).to(dev))
    b.set_params(w.params)
    x0, v0 = torch.from_numpy(w.x0).to(dev), torch.from_numpy(w.v0).to(dev)
    act = torch.from_numpy(w.act).to(dev)
    gx = torch.randn(E, n, 3, device=dev)
    dx, dv = torch.empty_like(gx), torch.empty_like(gx)
    da = torch.empty(S, E, T, device=dev)
    dp = torch.empty(E, 8, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    lib, h = b.lib, b.h
    from paper_2412_12089_amd import _capi as C

    def frame(backward=True):
        lib.mpm_fem_set_state(h, C.ptr(x0), C.ptr(v0))
        lib.mpm_fem_forward(h, S, C.ptr(act), C.MPM_FWD_RECORD if backward else 0)
        if backward:
            lib.mpm_fem_backward(h, C.ptr(gx), None, C.ptr(dx), C.ptr(dv), C.ptr(da), C.ptr(dp))

    def timed(backward):
        for _ in range(2):
            frame(backward)
        ms = []
        for _ in range(frames):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(b.stream)
            frame(backward)
            e1.record(b.stream)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        return float(np.mean(ms))

    fb_ms = timed(True)
    f_ms = timed(False)
    assert b.sync(raise_on_error=False) == C.MPM_OK, "non-finite FEM state"
    # HBM bytes of a frame: forward tape (S + 1 states of 24 B per node) and activations (4 B per element and
    # substep, read and kept); backward: the tape and activations read, the activation cotangents written
    frame_bytes = E * ((S + 1) * n * 24 * 2 + S * T * 4 * 4)
    out = {"workload": "soft_jumper", "envs": E, "nodes": n, "tets": T, "substeps": S,
           "fwd_bwd_ms_per_frame": fb_ms, "fwd_ms_per_frame": f_ms,
           "env_substeps_per_s": E * S / (fb_ms * 1e-3), "node_substeps_per_s": E * n * S / (fb_ms * 1e-3),
           "fwd_env_substeps_per_s": E * S / (f_ms * 1e-3), "frame_hbm_bytes": frame_bytes,
           "frame_hbm_gbs": frame_bytes / (fb_ms * 1e-3) / 1e9, "hbm_resident_bytes": b.memory_bytes()}
    b.close()
    return out


def rb_leg(n_envs, frames, dev):
    """The articulated rigid-body path on 13-link hands (a wrist and four
    three-link fingers with tip contacts): per 16-substep frame a recorded
    forward and its adjoint (cotangents of the initial state, the torques and
    the parameters), timed with HIP events on the library's stream."""
    import torch
    from paper_2412_12089_amd import _capi as C
    from paper_2412_12089_amd import rb_scenes as RS
    from paper_2412_12089_amd.rb import RbBatch
    w = RS.hand_batch(seed=9, n_envs=n_envs, substeps=16)
    E, N, S = w.n_envs, len(w.links), w.substeps
    b = RbBatch(w.links, E, S, w.dt, w.gravity, dev)
    b.set_params(w.params)
    q0, qd0 = torch.from_numpy(w.q0).to(dev), torch.from_numpy(w.qd0).to(dev)
    tau = torch.from_numpy(w.tau).to(dev)
    gq = torch.randn(E, N, device=dev)
    dq, dqd = torch.empty_like(gq), torch.empty_like(gq)
    dt = torch.empty(S, E, N, device=dev)
    dp = torch.empty(E, C.MPM_RB_PARAMS, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    lib, h = b.lib, b.h

    def frame(backward=True):
        lib.mpm_rb_set_state(h, C.ptr(q0), C.ptr(qd0))
        lib.mpm_rb_forward(h, S, C.ptr(tau), C.MPM_FWD_RECORD if backward else 0)
        if backward:
            lib.mpm_rb_backward(h, C.ptr(gq), None, C.ptr(dq), C.ptr(dqd), C.ptr(dt), C.ptr(dp))

    def timed(backward):
        for _ in range(2):
            frame(backward)
        ms = []
        for _ in range(frames):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(b.stream)
            frame(backward)
            e1.record(b.stream)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        return float(np.mean(ms))

    fb_ms = timed(True)
    f_ms = timed(False)
    assert b.sync(raise_on_error=False) == C.MPM_OK, "non-finite rigid-body state"
    out = {"workload": "hand", "envs": E, "links": N, "contacts": b.n_contacts, "substeps": S,
           "fwd_bwd_ms_per_frame": fb_ms, "fwd_ms_per_frame": f_ms,
           "env_substeps_per_s": E * S / (fb_ms * 1e-3), "joint_substeps_per_s": E * N * S / (fb_ms * 1e-3),
           "fwd_env_substeps_per_s": E * S / (f_ms * 1e-3), "hbm_resident_bytes": b.memory_bytes()}
    b.close()
    return out


def cpu_baseline(wl, substeps, n_envs, runs):
    """The FP64 oracle on a bounded sample: the first n_envs envs, `substeps`
    substeps each, forward + reverse; the median rate over `runs` runs."""
    import torch
    from oracle import mpm_oracle as O
    threads = torch.get_num_threads()
    specs = wl.envs[:max(1, n_envs)]
    rates, walls = [], []
    for _ in range(max(1, runs)):
        done, t_all = 0, 0.0
        for i, spec in enumerate(specs):
            env, prm, st = O.env_from_spec(spec)
            cot = O.linear_loss_cotangent(wl.loss_weights[i], spec.n_particles)
            t0 = time.perf_counter()
            O.rollout_vjp(env, prm, st, substeps, cot)   # forward (stores states) + per-substep reverse
            t_all += time.perf_counter() - t0
            done += spec.n_particles * substeps
        rates.append(done / t_all)
        walls.append(t_all)
    return {"value": float(np.median(rates)), "unit": "particle-substeps/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(specs)} env(s) of {wl.name} ({sum(s.n_particles for s in specs)} particles), "
                      f"{substeps} substeps fwd+bwd, median of {len(rates)} runs "
                      f"({', '.join(f'{t:.1f}' for t in walls)} s wall)"}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: environments never exchange data, so a multi-GPU run is "
              "independent single-GPU runs over disjoint env sets; run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2412_12089_amd import _capi, scenes
    from paper_2412_12089_amd.batch import Batch

    if args.fem_only:
        print(json.dumps(fem_leg(max(1, args.fem_envs), args.fem_frames, torch.device("cuda:0"))), flush=True)
        return
    if args.rb_only:
        print(json.dumps(rb_leg(max(1, args.rb_envs), args.rb_frames, torch.device("cuda:0"))), flush=True)
        return
    wl = scenes.WORKLOADS[args.workload]()
    S, K = wl.substeps, wl.ckpt_every
    envs = wl.envs
    N = sum(e.n_particles for e in envs)
    dev = torch.device("cuda:0")
    x0, w = inputs(wl, dev)
    fixed = dict(kv.split("=") for kv in args.set.split(",") if kv)
    progress(f"{wl.name}: {len(envs)} envs, {N} particles, {S} substeps; batch created, autotuning")
    b, tuned, tune_s = tuned_batch(wl, dev, args, fixed)
    progress(f"options {tuned}; timing {args.steps} steps")
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
               "g2p2g": b.get_option(_capi.OPT_FUSE) * (2 if b.get_option(_capi.OPT_P2G) == 3 else 1),
               "adj_pair": b.get_option(_capi.OPT_FUSE_ADJ)}
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
    # whole step against the method's bytes: 672 B per particle-substep fwd+bwd, 96/K B of
    # checkpoints, 28 + 56 B per touched node and substep
    step_bytes = N * S * (672 + 96.0 / K) + nodes * S * (28 + 56)

    progress(f"{np.mean(ms):.1f} ms per step; per-env mode next")
    plain = None
    if args.plain_steps > 0:
        bp = Batch(envs, max_substeps=S, ckpt_every=K, mode="plain", device=dev)
        pms = run_steps(bp, x0, w, S, args.plain_steps, 1)
        bp.close()
        plain = N * S / (float(np.mean(pms)) * 1e-3)

    extra = {}
    for name in [n for n in args.extra.split(",") if n and n != wl.name]:
        progress(f"workload {name}")
        extra[name] = extra_workload(name, dev, args)

    fem = None
    if args.fem_envs > 0:
        progress(f"FEM leg: {args.fem_envs} jumpers")
        fem = fem_leg(args.fem_envs, args.fem_frames, dev)

    rb = None
    if args.rb_envs > 0:
        progress(f"rigid-body leg: {args.rb_envs} hands")
        rb = rb_leg(args.rb_envs, args.rb_frames, dev)

    serving = None
    if args.serve_seconds > 0:
        progress(f"serving a {args.serve_seconds:.0f} s Poisson stream")
        serving = serving_leg(args.serve_seconds, args.serve_rate, args.serve_slots, dev)
    if not args.no_cpu_baseline:
        progress("oracle CPU baseline")
    cpu = None if args.no_cpu_baseline else cpu_baseline(wl, args.cpu_substeps, args.cpu_envs, args.cpu_runs)
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
        "step_alg_bytes": step_bytes,
        "step_alg_gbs": step_bytes / (step_ms * 1e-3) / 1e9,
        "kernel_ms": {k: v[0] for k, v in kt.items()},
        "kernel_launches_per_step": {k: v[1] for k, v in kt.items()},
        "roofline": {"bound": "hbm", "kernel": symbol, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "alg_bytes_per_launch": alg_bytes, "touched_nodes": nodes, "kernel_ms": dom_ms},
        "workloads": extra,
        "fem": fem,
        "rigid": rb,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
