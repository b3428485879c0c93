"""Writes fullsize_oracle.npz: FP64 oracle results on the full-size workloads
that are too slow to recompute inside a GPU test.

* dam break (16 envs x 200,000 Tait particles, 96^3, 100 substeps): env 0,
  the whole horizon, forward and the reverse pass of L = sum_p x_p . w_p;
* uneven mixed (64 envs, 64^3, 50 substeps): 8 envs stratified by material
  (neo-Hookean and von Mises: the smallest, median and largest env;
  Tait fluid: the smallest and largest), forward and reverse pass.

For each env a seeded sample of particles is stored (the final x, v, C, F and
the initial-state cotangents, float32) together with the env's parameter
cotangent row (float64). Only the oracle and the seeded scene generators are
called. Run from the repository root:

    python tests/golden/make_fullsize_oracle.py
"""
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import mpm_oracle as O  # noqa: E402
from paper_2412_12089_amd import scenes  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize_oracle.npz")
SAMPLE_SEED = 2412


def stratified_uneven(wl):
    """8 envs of the uneven workload: per material, envs at the size extremes (and median)."""
    picks = []
    for mat, k in ((scenes.NEOHOOKEAN, 3), (scenes.VONMISES, 3), (scenes.FLUID_TAIT, 2)):
        ids = sorted((e.n_particles, i) for i, e in enumerate(wl.envs) if e.material == mat)
        at = [0, len(ids) - 1] if k == 2 else [0, len(ids) // 2, len(ids) - 1]
        picks += [ids[j][1] for j in at]
    return picks


def sample_indices(N, k, salt):
    rng = np.random.Generator(np.random.PCG64([SAMPLE_SEED, salt]))
    return np.sort(rng.choice(N, size=min(k, N), replace=False))


def run(tag, wl, i, k, out):
    spec = wl.envs[i]
    S = wl.substeps
    t0 = time.perf_counter()
    env, prm, st = O.env_from_spec(spec)
    (x, v, C, F), oob = O.rollout(env, prm, st, S)
    assert not oob
    cot = O.linear_loss_cotangent(wl.loss_weights[i], spec.n_particles)
    g, gp = O.rollout_vjp(env, prm, st, S, cot)
    idx = sample_indices(spec.n_particles, k, i)
    key = f"{tag}_{i}"
    out[key + "_idx"] = idx.astype(np.int64)
    for name, a in zip(("x", "v", "C", "F"), (x, v, C, F)):
        out[f"{key}_{name}"] = a.numpy()[idx].astype(np.float32)
    for name, a in zip(("dx0", "dv0", "dC0", "dF0"), g):
        out[f"{key}_{name}"] = a.numpy()[idx].astype(np.float32)
    out[key + "_dparams"] = O.param_cotangent_row(gp)
    out[key + "_meta"] = np.array([spec.n_particles, S, spec.material], dtype=np.int64)
    print(f"{key}: {spec.n_particles} particles ({scenes.MATERIAL_NAMES[spec.material]}), {S} substeps, "
          f"{time.perf_counter() - t0:.0f} s", flush=True)


def main():
    out = {}
    dam = scenes.dam_break()
    run("dam_break", dam, 0, 2048, out)
    uneven = scenes.uneven_mixed()
    picks = stratified_uneven(uneven)
    out["uneven_mixed_envs"] = np.array(picks, dtype=np.int64)
    for i in picks:
        run("uneven_mixed", uneven, i, 512, out)
    np.savez_compressed(OUT, **out)
    print(f"wrote {OUT} ({os.path.getsize(OUT) / 1e6:.2f} MB)")


if __name__ == "__main__":
    main()
