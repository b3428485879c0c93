"""A minimal SAPO learner (the paper's Algorithm 1, Section 4) on a synthetic
MPM manipulation task run by the batched differentiable simulator.

SAPO is maximum-entropy first-order model-based RL: the actor maximizes the
entropy-augmented H-step return plus the soft value of the last state, with
gradients taken analytically through the simulation (here: MPMRollout chained
over env steps, the box pusher's per-substep velocities as actions, rewards
from the device-side moments); C critics (no target networks) learn soft
values by TD(lambda) on soft returns, the minimum of the critics forming the
targets and their mean entering the actor's return; the temperature is tuned
to a target entropy of -dim(A)/2 and the entropy is normalized by it. Design
choices follow Section 4.2: squashed-Normal policy with state-dependent
variance, LayerNorm + SiLU MLPs, AdamW, gradient norm clipping at 0.5.

`HandEnv` and `JumperEnv` are tasks on the articulated rigid-body and the
tetrahedral FEM paths (see their docstrings). The first task (`PushTask`) stands in for the paper's manipulation scenes, whose
assets are not available: E envs, each a neo-Hookean block of dough with a box
pusher beside it; an action a in [-1, 1]^3 sets the box velocity
(max_speed * a) for the substeps of one env step; the reward is the progress of
the dough's centre of mass along +x (from a subsample, via the device-side
moments) minus a small action cost. Observations: centre of mass, mean
velocity, height variance of the subsample and the box centre.
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np
import torch
import torch.nn as nn

from . import observe, scenes
from .batch import Batch, rollout


@dataclasses.dataclass
class PushTask:
    n_envs: int = 8
    n: int = 32
    n_particles: int = 1500
    substeps: int = 20          # simulation substeps per env step
    dt: float = 2e-4
    max_speed: float = 2.0      # box speed at |a| = 1 (m/s)
    episode: int = 6            # env steps per episode
    subsample: int = 4          # every subsample-th particle enters the observation and reward
    reward_scale: float = 100.0
    action_cost: float = 1e-3
    seed: int = 0


class PushEnv:
    obs_dim = 10
    act_dim = 3

    def __init__(self, task: PushTask, device=None):
        self.task = task
        self.device = device or torch.device("cuda:0")
        rng = np.random.Generator(np.random.PCG64(task.seed))
        specs = []
        for _ in range(task.n_envs):
            lo = np.array([0.32, 0.42, 0.16]) + rng.uniform(-0.02, 0.02, size=3)
            side = np.array([0.12, 0.12, 0.12])
            x = scenes.uniform_points(rng, lo, side, task.n_particles)
            C, F = scenes._rest_state(task.n_particles)
            box = scenes.BoxCollider(center=(float(lo[0] - 0.045), float(lo[1] + 0.06), float(lo[2] + 0.06)),
                                     half=(0.03, 0.05, 0.05), velocity=(0.0, 0.0, 0.0),
                                     alpha=2.0 * task.n, mu_b=0.5)
            specs.append(scenes.EnvSpec(n=task.n, dt=task.dt, material=scenes.NEOHOOKEAN, E=5e3, nu=0.3, rho=1e3,
                                        Vp=float(np.prod(side)) / task.n_particles, x=x,
                                        v=np.zeros_like(x), C=C, F=F, collider=box))
        self.specs = specs
        self.batch = Batch(specs, max_substeps=task.substeps, ckpt_every=task.substeps, mode="batched",
                           device=self.device)
        self.params = torch.tensor(np.stack([e.params() for e in specs]), dtype=torch.float64)
        self.w = observe.subsample_weights(self.batch, task.subsample)
        cat = lambda k: torch.from_numpy(np.concatenate([getattr(e, k) for e in specs], axis=0)).to(self.device)
        self.init_state = tuple(cat(k) for k in ("x", "v", "C", "F"))
        self.init_centers = torch.tensor([e.collider.center for e in specs], dtype=torch.float32)

    def reset(self):
        return tuple(t.clone() for t in self.init_state), self.init_centers.clone()

    def stats(self, state):
        m = observe.moments(self.batch, state[0], state[1], self.w)
        return observe.center_of_mass(m), observe.mean_velocity(m), observe.height_variance(m)

    def obs(self, state, centers):
        com, vbar, var_z = self.stats(state)
        o = torch.cat([(com - 0.4) * 10.0, vbar, var_z[:, None] * 1e3, (centers.to(com.device).double() - 0.4) * 10.0], 1)
        return o.float()

    def step(self, state, centers, a):
        """One env step, differentiable in state, centers and a [E, 3] (on the CPU, float32)."""
        T = self.task
        vel = (T.max_speed * a)[:, None, :].expand(-1, T.substeps, -1).contiguous()
        com0 = self.stats(state)[0][:, 0]
        nxt = rollout(self.batch, T.substeps, *state, self.params, vel, centers)
        new_centers = centers + (T.dt * T.substeps * T.max_speed) * a
        com1 = self.stats(nxt)[0][:, 0]
        r = T.reward_scale * (com1 - com0).float().cpu() - T.action_cost * (a ** 2).sum(1)
        return nxt, new_centers, r

    def close(self):
        self.batch.close()


@dataclasses.dataclass
class SqueezeTask:
    n_envs: int = 8
    n: int = 32
    n_particles: int = 1500
    substeps: int = 20          # simulation substeps per env step
    dt: float = 2e-4
    max_speed: float = 1.5      # jaw speed at |a| = 1 (m/s)
    subsample: int = 4          # every subsample-th particle enters the observation and reward
    reward_scale: float = 300.0
    action_cost: float = 1e-3
    seed: int = 0


class SqueezeEnv:
    """A soft cube between two jaws (two box colliders of one env, slots 0 and
    1), each driven by its own velocity: the actions are both jaws' velocities
    and the reward is the rise of the cube's centre of mass (squeezing it
    makes it bulge up, dragging it lifts it by friction)."""
    obs_dim = 13
    act_dim = 6

    def __init__(self, task: SqueezeTask, device=None):
        self.task = task
        self.device = device or torch.device("cuda:0")
        rng = np.random.Generator(np.random.PCG64(task.seed))
        specs = []
        for _ in range(task.n_envs):
            lo = np.array([0.42, 0.42, 0.16]) + rng.uniform(-0.02, 0.02, size=3)
            side = np.array([0.12, 0.12, 0.12])
            x = scenes.uniform_points(rng, lo, side, task.n_particles)
            C, F = scenes._rest_state(task.n_particles)
            jaw = lambda cx: scenes.BoxCollider(center=(float(cx), float(lo[1] + 0.06), float(lo[2] + 0.06)),
                                                half=(0.03, 0.07, 0.07), velocity=(0.0, 0.0, 0.0),
                                                alpha=2.0 * task.n, mu_b=0.8)
            specs.append(scenes.EnvSpec(n=task.n, dt=task.dt, material=scenes.NEOHOOKEAN, E=5e3, nu=0.3, rho=1e3,
                                        Vp=float(np.prod(side)) / task.n_particles, x=x, v=np.zeros_like(x), C=C,
                                        F=F, collider=jaw(lo[0] - 0.04), more_colliders=(jaw(lo[0] + 0.16),)))
        self.specs = specs
        self.batch = Batch(specs, max_substeps=task.substeps, ckpt_every=task.substeps, mode="batched",
                           device=self.device)
        self.params = torch.tensor(np.stack([e.params() for e in specs]), dtype=torch.float64)
        self.w = observe.subsample_weights(self.batch, task.subsample)
        cat = lambda k: torch.from_numpy(np.concatenate([getattr(e, k) for e in specs], axis=0)).to(self.device)
        self.init_state = tuple(cat(k) for k in ("x", "v", "C", "F"))
        self.init_centers = torch.tensor([[e.collider.center, e.more_colliders[0].center] for e in specs],
                                         dtype=torch.float32)

    def reset(self):
        return tuple(t.clone() for t in self.init_state), self.init_centers.clone()

    def stats(self, state):
        m = observe.moments(self.batch, state[0], state[1], self.w)
        return observe.center_of_mass(m), observe.mean_velocity(m), observe.height_variance(m)

    def obs(self, state, centers):
        com, vbar, var_z = self.stats(state)
        jaws = (centers.to(com.device).double().reshape(-1, 6) - 0.4) * 10.0
        return torch.cat([(com - 0.4) * 10.0, vbar, var_z[:, None] * 1e3, jaws], 1).float()

    def step(self, state, centers, a):
        """One env step, differentiable in state, centers [E, 2, 3] and a [E, 6] (on the CPU, float32)."""
        T = self.task
        a2 = a.reshape(-1, 2, 3)
        vel = (T.max_speed * a2)[:, :, None, :].expand(-1, -1, T.substeps, -1).contiguous()
        z0 = self.stats(state)[0][:, 2]
        nxt = rollout(self.batch, T.substeps, *state, self.params, vel, centers)
        new_centers = centers + (T.dt * T.substeps * T.max_speed) * a2
        z1 = self.stats(nxt)[0][:, 2]
        r = T.reward_scale * (z1 - z0).float().cpu() - T.action_cost * (a ** 2).sum(1)
        return nxt, new_centers, r

    def close(self):
        self.batch.close()


@dataclasses.dataclass
class HandTask:
    n_envs: int = 16
    substeps: int = 16          # rigid-body substeps per env step (one 1/60 s frame)
    max_torque: float = 1e-2    # joint torque at |a| = 1 (N m)
    reward_scale: float = 10.0
    action_cost: float = 1e-3
    seed: int = 0


class HandEnv:
    """A second task, on the articulated rigid-body path: E 13-link hands
    (`rb_scenes.hand_batch`, finger tips over a ground) start at random joint
    angles and speeds; an action a in [-1, 1]^13 sets the joint torques
    (max_torque * a) for the substeps of one env step; the reward is the
    progress of the joints toward a curled target pose (mean squared angle
    error, wrist 0.3 rad, finger joints 0.8 rad) minus a small action cost.
    Observations: the angle errors and the joint speeds. Env steps are chained
    `RBRollout` calls, so the actor's gradient runs through the rigid-body
    adjoint."""
    act_dim = 13
    obs_dim = 26

    def __init__(self, task: HandTask, device=None):
        from . import rb_scenes
        from .rb import RbBatch
        self.task = task
        self.device = device or torch.device("cuda:0")
        w = rb_scenes.hand_batch(seed=task.seed, n_envs=task.n_envs, substeps=task.substeps)
        self.batch = RbBatch(w.links, task.n_envs, task.substeps, w.dt, w.gravity, self.device)
        self.params = torch.from_numpy(w.params)
        self.init_state = (torch.from_numpy(w.q0).to(self.device), torch.from_numpy(w.qd0).to(self.device))
        tgt = np.full(len(w.links), 0.8, dtype=np.float32)
        tgt[0] = 0.3
        self.target = torch.from_numpy(tgt).to(self.device)
        self.none = torch.zeros(task.n_envs, 1)

    def reset(self):
        return tuple(t.clone() for t in self.init_state), self.none

    def obs(self, state, _):
        q, qd = state
        return torch.cat([q - self.target, 0.1 * qd], 1).float()

    def step(self, state, _, a):
        """One env step, differentiable in state and a [E, 13] (on the CPU, float32)."""
        from .rb import rollout
        T = self.task
        tau = (T.max_torque * a.to(self.device))[None].expand(T.substeps, -1, -1).contiguous()
        d0 = ((state[0] - self.target) ** 2).mean(1)
        nxt = rollout(self.batch, T.substeps, state[0], state[1], tau, self.params)
        d1 = ((nxt[0] - self.target) ** 2).mean(1)
        r = T.reward_scale * (d0 - d1).float().cpu() - T.action_cost * (a ** 2).sum(1)
        return nxt, self.none, r

    def close(self):
        self.batch.close()


@dataclasses.dataclass
class JumperTask:
    n_envs: int = 16
    substeps: int = 80          # FEM substeps per env step (one 1/60 s frame)
    act_scale: float = 0.3      # element activation at |a| = 1
    reward_scale: float = 300.0
    action_cost: float = 1e-3
    seed: int = 0


class JumperEnv:
    """A third task, on the tetrahedral FEM path: E soft jumpers
    (`fem_scenes.soft_jumper`) standing on the ground; the elements form eight
    muscle groups (the octants of the rest shape about its centre), and an
    action a in [-1, 1]^8 sets every element's activation to act_scale times
    its group's entry for the substeps of one env step; the reward is the
    rise plus the forward (+x) progress of the mean node position (a jump;
    the ground's viscous friction is too weak to walk on) minus a small
    action cost.
    Observations: the mean node position relative to the start and the mean
    node velocity. Env steps are chained `FEMRollout` calls."""
    act_dim = 8
    obs_dim = 6

    def __init__(self, task: JumperTask, device=None):
        from . import fem_scenes
        from .fem import FemBatch
        self.task = task
        self.device = device or torch.device("cuda:0")
        w = fem_scenes.soft_jumper(seed=task.seed, n_envs=task.n_envs, substeps=task.substeps)
        n = w.X.shape[1]
        self.batch = FemBatch(w.tets, task.n_envs, n, task.substeps, w.dt, w.gravity, self.device)
        self.batch.set_rest(torch.from_numpy(w.X).to(self.device))
        self.params = torch.from_numpy(w.params)
        self.init_state = (torch.from_numpy(w.x0).to(self.device), torch.from_numpy(w.v0).to(self.device))
        X0 = w.X[0].astype(np.float64)
        cen = X0[w.tets].mean(1)                       # element centroids of env 0's rest shape
        mid = X0.mean(0)
        grp = ((cen[:, 0] > mid[0]) * 4 + (cen[:, 1] > mid[1]) * 2 + (cen[:, 2] > mid[2])).astype(np.int64)
        onehot = np.zeros((w.tets.shape[0], 8), dtype=np.float32)
        onehot[np.arange(len(grp)), grp] = 1.0
        self.groups = torch.from_numpy(onehot).to(self.device)     # [T, 8]
        self.start = self.init_state[0].mean(1)
        self.none = torch.zeros(task.n_envs, 1)

    def reset(self):
        return tuple(t.clone() for t in self.init_state), self.none

    def obs(self, state, _):
        x, v = state
        return torch.cat([10.0 * (x.mean(1) - self.start), v.mean(1)], 1).float()

    def step(self, state, _, a):
        """One env step, differentiable in state and a [E, 8] (on the CPU, float32)."""
        from .fem import rollout
        T = self.task
        act = (T.act_scale * a.to(self.device)) @ self.groups.T                  # [E, T]
        act = act[None].expand(T.substeps, -1, -1).contiguous()
        c0 = (state[0][:, :, 0] + state[0][:, :, 2]).mean(1)
        nxt = rollout(self.batch, T.substeps, state[0], state[1], act, self.params)
        c1 = (nxt[0][:, :, 0] + nxt[0][:, :, 2]).mean(1)
        r = T.reward_scale * (c1 - c0).float().cpu() - T.action_cost * (a ** 2).sum(1)
        return nxt, self.none, r

    def close(self):
        self.batch.close()


def td_lambda_targets(r, v_next, gamma: float, lam: float):
    """lambda-returns of an H-step window (TD(lambda) of the SHAC/SAPO critic):
    r [H, E] the (soft) rewards, v_next [H, E] the value of s_{t+1}; returns
    [H, E], G_t = r_t + gamma ((1 - lam) V(s_{t+1}) + lam G_{t+1}) with
    G_{H-1} = r_{H-1} + gamma V(s_H), which is the weighted average of the
    value-bootstrapped k-step returns."""
    H = r.shape[0]
    out = torch.empty_like(r)
    nxt = None
    for t in reversed(range(H)):
        nxt = r[t] + gamma * v_next[t] if t == H - 1 else r[t] + gamma * ((1.0 - lam) * v_next[t] + lam * nxt)
        out[t] = nxt
    return out


def mlp(i, o, width=64):
    return nn.Sequential(nn.Linear(i, width), nn.LayerNorm(width), nn.SiLU(),
                         nn.Linear(width, width), nn.LayerNorm(width), nn.SiLU(), nn.Linear(width, o))


class Actor(nn.Module):
    """Squashed Normal with state-dependent variance: a = tanh(u), u ~ N(mu(s), sigma(s)^2)."""

    def __init__(self, obs_dim, act_dim):
        super().__init__()
        self.net = mlp(obs_dim, 2 * act_dim)
        self.act_dim = act_dim

    def forward(self, obs):
        mu, log_std = self.net(obs).split(self.act_dim, -1)
        std = log_std.clamp(-5.0, 2.0).exp()
        u = mu + std * torch.randn_like(mu)                      # reparameterized sample
        a = torch.tanh(u)
        logp = (-0.5 * ((u - mu) / std) ** 2 - std.log() - 0.5 * math.log(2 * math.pi)).sum(-1)
        logp = logp - torch.log(1.0 - a ** 2 + 1e-6).sum(-1)     # change of variables through tanh
        return a, logp


class SAPO:
    def __init__(self, env, horizon: int = 6, gamma: float = 0.99, lam: float = 0.95, n_critics: int = 2,
                 critic_iters: int = 8, lr_actor: float = 2e-3, lr_critic: float = 2e-3, lr_alpha: float = 5e-3,
                 seed: int = 0):
        torch.manual_seed(seed)
        self.env = env
        self.H, self.gamma, self.lam, self.critic_iters = horizon, gamma, lam, critic_iters
        self.actor = Actor(env.obs_dim, env.act_dim)
        self.critics = nn.ModuleList([mlp(env.obs_dim, 1) for _ in range(n_critics)])
        betas = (0.7, 0.95)
        self.opt_a = torch.optim.AdamW(self.actor.parameters(), lr=lr_actor, betas=betas)
        self.opt_c = torch.optim.AdamW(self.critics.parameters(), lr=lr_critic, betas=betas)
        self.log_alpha = torch.zeros((), requires_grad=True)
        self.opt_alpha = torch.optim.AdamW([self.log_alpha], lr=lr_alpha, betas=betas, weight_decay=0.0)
        self.target_entropy = -env.act_dim / 2.0
        self.history = []

    def values(self, obs):
        return torch.stack([c(obs).squeeze(-1) for c in self.critics])   # [C, E]

    def iteration(self):
        """One Algorithm 1 iteration over an episode of H env steps (reset at its start)."""
        env, H, g = self.env, self.H, self.gamma
        t0 = time.perf_counter()
        state, centers = env.reset()
        alpha = self.log_alpha.exp().detach()
        hbar = abs(self.target_entropy)
        obs = env.obs(state, centers).cpu()
        ret = torch.zeros(env.task.n_envs)
        buf_obs, buf_r, buf_h, buf_v = [], [], [], []
        for t in range(H):
            a, logp = self.actor(obs)
            h = -logp                                               # single-sample entropy estimate
            hn = (h + hbar) / (2.0 * hbar)                          # normalized entropy
            state, centers, r = env.step(state, centers, a)
            obs_next = env.obs(state, centers).cpu()
            ret = ret + (g ** t) * (r + alpha * hn)
            buf_obs.append(obs.detach()); buf_r.append(r.detach()); buf_h.append(hn.detach())
            buf_v.append(self.values(obs_next.detach()).detach())
            obs = obs_next
        v_last = self.values(obs).mean(0)                           # mean of the critics for the actor
        actor_loss = -(ret + (g ** H) * v_last).mean() / H
        self.opt_a.zero_grad()
        actor_loss.backward()                                       # analytic gradients through the simulator
        gnorm = float(nn.utils.clip_grad_norm_(self.actor.parameters(), 0.5))
        self.opt_a.step()
        # temperature: alpha <- alpha - eta d/d(alpha)[alpha (h - target)]
        h_raw = torch.stack([(hn * 2.0 * hbar - hbar) for hn in buf_h])
        alpha_loss = (self.log_alpha.exp() * (h_raw - self.target_entropy)).mean()
        self.opt_alpha.zero_grad()
        alpha_loss.backward()
        self.opt_alpha.step()
        # TD(lambda) targets on soft returns with the minimum of the critics
        vmin = torch.stack([v.min(0).values for v in buf_v])        # V(s_{t+1}), t = 0..H-1
        soft_r = torch.stack(buf_r) + alpha * torch.stack(buf_h)
        targets = td_lambda_targets(soft_r, vmin, g, self.lam)
        X = torch.cat(buf_obs)
        Y = targets.reshape(-1)
        for _ in range(self.critic_iters):
            closs = sum(((c(X).squeeze(-1) - Y) ** 2).mean() for c in self.critics)
            self.opt_c.zero_grad()
            closs.backward()
            nn.utils.clip_grad_norm_(self.critics.parameters(), 0.5)
            self.opt_c.step()
        rec = {"return": torch.stack(buf_r).sum(0).mean().item(), "actor_loss": actor_loss.detach().item(),
               "critic_loss": closs.detach().item(), "alpha": self.log_alpha.exp().detach().item(), "grad_norm": gnorm,
               "entropy": h_raw.mean().item(), "seconds": time.perf_counter() - t0}
        self.history.append(rec)
        return rec
