"""Host sequencing of the learned proposal: log plain-walker states, train the
network, and hold its buffers.

Every computation is a call into liblabs.so (labs_learned_walk for the log,
labs_mlp_train_step for training, labs_mlp_forward for scoring); this module
only allocates device buffers, keeps the Adam step count and walks the log in
batches.  The log is step-major, so a contiguous batch holds states of many
different walkers.
"""
from __future__ import annotations

from . import labs


class Network:
    """FP32 master parameters, their bf16 copy, Adam moments and a gradient
    buffer for the network of width `hidden` at sequence length L."""

    def __init__(self, L: int, init: dict, hidden: int = 256, device="cuda"):
        torch = labs._torch()
        self.L, self.hidden = L, hidden
        self.lay = labs.mlp_layout(L, hidden)
        blob = labs.mlp_blob_from_dict(self.lay, init)
        self.params = torch.from_numpy(blob).to(device)
        self.params_bf16 = torch.empty(self.lay.n_params, dtype=torch.bfloat16, device=device)
        labs.mlp_cast(self.lay, self.params, self.params_bf16)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grads = torch.zeros_like(self.params)
        self.t = 0
        self._ws = None
        self._loss = torch.zeros(1, dtype=torch.float32, device=device)

    def clone(self) -> "Network":
        other = object.__new__(Network)
        other.__dict__.update(self.__dict__)
        for k in ("params", "params_bf16", "m", "v", "grads", "_loss"):
            setattr(other, k, getattr(self, k).clone())
        other._ws = None
        return other

    def train_step(self, seqs, mask, labels, lr=1e-3):
        """One Adam step on a batch of logged records; returns the device loss."""
        self.t += 1
        _, self._ws = labs.mlp_train_step(self.lay, self.params, self.params_bf16, self.grads, self.m,
                                          self.v, self.t, seqs, mask, labels, lr=lr,
                                          workspace=self._ws, loss=self._loss)
        return self._loss

    def logits(self, seqs):
        X = labs.mlp_features(self.L, seqs)
        return labs.mlp_forward(self.lay, self.params, self.params_bf16, X)

    def proposer_args(self) -> dict:
        return dict(mode=labs.PROPOSE_MLP, hidden=self.hidden, params=self.params,
                    params_bf16=self.params_bf16)


def log_plain(L: int, p: int, steps: int, tenure_lo: int, tenure_hi: int, seed: int, n_walkers: int,
              log_every: int, walker_begin: int = 0, device="cuda"):
    """States, admissible masks and moves of plain walkers (every step a full exact
    scan), one record per walker every `log_every` steps, step-major."""
    r = labs.learned_walk(L, p, steps, tenure_lo, tenure_hi, seed, n_walkers,
                          mode=labs.PROPOSE_RANDOM, top_m=1, fallback_every=1, log_every=log_every,
                          walker_begin=walker_begin, device=device)
    return r["log_seqs"], r["log_mask"], r["log_label"]


def train(net: Network, seqs, mask, labels, batch: int = 4096, epochs: float = 1.0, lr: float = 1e-3,
          report_every: int = 0):
    """Adam over contiguous batches of the log for `epochs` passes; returns the
    (step, loss) pairs read back every `report_every` steps (0: first and last)."""
    n = seqs.shape[0]
    per_epoch = max(1, n // batch)
    total = max(1, int(round(epochs * per_epoch)))
    out = []
    for s in range(total):
        b = (s % per_epoch) * batch
        loss = net.train_step(seqs[b:b + batch], mask[b:b + batch], labels[b:b + batch], lr=lr)
        if (report_every and (s + 1) % report_every == 0) or s in (0, total - 1):
            out.append((net.t, float(loss.item())))
    return out
