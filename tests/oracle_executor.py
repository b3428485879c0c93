"""A server executor that runs the FP64 oracle on the CPU (scheduler tests only)."""
import numpy as np
import torch

from oracle import mpm_oracle as O


class OracleExecutor:
    def __init__(self, n_slots, n_cap=64, N_cap=100_000):
        self.n_slots = n_slots
        self.capacity = (n_cap, N_cap)
        self.slots = [None] * n_slots
        self.calls = []
        self.errs = {}

    def load(self, slot, spec):
        env, prm, st = O.env_from_spec(spec)
        self.slots[slot] = dict(env=env, prm=prm, st=st, rec=None)

    def unload(self, slot):
        self.slots[slot] = None

    def snapshot(self, slot):
        return tuple(t.clone() for t in self.slots[slot]["st"])

    def restore(self, slot, snap):
        self.slots[slot]["st"] = tuple(t.clone() for t in snap)

    def forward(self, counts, record):
        self.calls.append(("fwd_rec" if record else "fwd", list(counts)))
        for s, k in enumerate(counts):
            if k and self.slots[s] is not None:
                d = self.slots[s]
                if record:
                    d["rec"] = (d["st"], k)
                d["st"], oob = O.rollout(d["env"], d["prm"], d["st"], k)
                bits = (0 if all(bool(torch.isfinite(t).all()) for t in d["st"]) else 1) | (2 if oob else 0)
                if bits:
                    self.errs[s] = self.errs.get(s, 0) | bits

    def loss_cotangent(self, req):
        return O.linear_loss_cotangent(req.loss_weights, req.env.n_particles)

    def backward(self, cots):
        out = {}
        for s, c in cots.items():
            d = self.slots[s]
            st0, k = d["rec"]
            g, gp = O.rollout_vjp(d["env"], d["prm"], st0, k, c)
            out[s] = (g, O.param_cotangent_row(gp))
        return out

    def read(self, slot):
        return self.slots[slot]["st"]

    def sync(self):
        out, self.errs = self.errs, {}
        return out
