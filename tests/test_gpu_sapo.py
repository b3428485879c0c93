"""The minimal SAPO learner on the push task: analytic policy gradients through
chained differentiable rollouts, collider actions and device-side rewards."""
import math

import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def test_sapo_improves_the_push_return():
    from paper_2412_12089_amd.sapo import SAPO, PushEnv, PushTask
    env = PushEnv(PushTask(n_envs=16, n_particles=1200))
    try:
        agent = SAPO(env, horizon=6, seed=0)
        recs = [agent.iteration() for _ in range(16)]
    finally:
        env.close()
    for i, r in enumerate(recs):
        print(f"[gpu-sapo] iteration {i}: " + " ".join(f"{k} {v:.4g}" for k, v in r.items()), flush=True)
        assert all(math.isfinite(v) for v in r.values())
    assert all(r["grad_norm"] > 0 for r in recs)
    first = np.mean([r["return"] for r in recs[:2]])
    last = np.mean([r["return"] for r in recs[-4:]])
    assert last > 1.5 * first + 0.1, (first, last)
    assert recs[-1]["alpha"] < recs[0]["alpha"]   # entropy above target: the temperature falls


def test_sapo_improves_the_hand_return():
    """The same learner on the rigid-body hand task: analytic policy gradients
    through chained rigid-body rollouts (the torques are the actions)."""
    from paper_2412_12089_amd.sapo import SAPO, HandEnv, HandTask
    env = HandEnv(HandTask(n_envs=16))
    try:
        agent = SAPO(env, horizon=8, seed=0)
        recs = [agent.iteration() for _ in range(20)]
    finally:
        env.close()
    for i, r in enumerate(recs):
        print(f"[gpu-sapo] hand iteration {i}: " + " ".join(f"{k} {v:.4g}" for k, v in r.items()), flush=True)
        assert all(math.isfinite(v) for v in r.values())
    assert all(r["grad_norm"] > 0 for r in recs)
    first = np.mean([r["return"] for r in recs[:2]])
    last = np.mean([r["return"] for r in recs[-4:]])
    assert last > first + 0.5 * abs(first) + 0.05, (first, last)


def test_sapo_improves_the_jumper_return():
    """The same learner on the FEM jumper task: analytic policy gradients
    through chained FEM rollouts (grouped element activations are the actions)."""
    from paper_2412_12089_amd.sapo import SAPO, JumperEnv, JumperTask
    env = JumperEnv(JumperTask(n_envs=16))
    try:
        agent = SAPO(env, horizon=6, seed=0)
        recs = [agent.iteration() for _ in range(20)]
    finally:
        env.close()
    for i, r in enumerate(recs):
        print(f"[gpu-sapo] jumper iteration {i}: " + " ".join(f"{k} {v:.4g}" for k, v in r.items()), flush=True)
        assert all(math.isfinite(v) for v in r.values())
    assert all(r["grad_norm"] > 0 for r in recs)
    first = np.mean([r["return"] for r in recs[:2]])
    last = np.mean([r["return"] for r in recs[-4:]])
    assert last > first + 0.5 * abs(first) + 0.05, (first, last)


def test_sapo_improves_the_squeeze_return():
    """The learner on a two-jaw task: the actions drive two colliders of one
    env through the autograd Function's per-slot actions and centers."""
    from paper_2412_12089_amd.sapo import SAPO, SqueezeEnv, SqueezeTask
    env = SqueezeEnv(SqueezeTask(n_envs=16, n_particles=1200))
    try:
        agent = SAPO(env, horizon=6, seed=0)
        recs = [agent.iteration() for _ in range(16)]
    finally:
        env.close()
    for i, r in enumerate(recs):
        print(f"[gpu-sapo] squeeze iteration {i}: " + " ".join(f"{k} {v:.4g}" for k, v in r.items()), flush=True)
        assert all(math.isfinite(v) for v in r.values())
    assert all(r["grad_norm"] > 0 for r in recs)
    first = np.mean([r["return"] for r in recs[:2]])
    last = np.mean([r["return"] for r in recs[-4:]])
    assert last > first + 0.5 * abs(first) + 0.05, (first, last)
