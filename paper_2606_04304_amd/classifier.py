"""Training loop and scoring for the candidate classifier (nbsi_net_*): class-balanced mini-batch
Adam steps, batched scores, the operating point and precision / recall of accepted candidates.
Orchestration only: every numerical step of the network runs in libnbsi.  (The training data,
stamps of the detector's candidates over dumps with injected tones, RFI and spikes, come from
the synthetic-input package, synth.injections.)
"""
from __future__ import annotations

import numpy as np

from . import Net


def _torch():
    import torch
    return torch


def balanced_index(labels: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    """Every negative once and the positives repeated to about as many, shuffled."""
    pos = np.flatnonzero(labels > 0.5)
    neg = np.flatnonzero(labels <= 0.5)
    reps = max(1, int(round(len(neg) / max(1, len(pos)))))
    idx = np.concatenate([neg] + [pos] * reps)
    rng.shuffle(idx)
    return idx.astype(np.int32)


def train(net: Net, stamps, labels: np.ndarray, epochs: int, batch: int, lr: float, seed: int, log=None):
    """Adam on mini-batches of a class-balanced index list; returns the mean loss per epoch."""
    torch = _torch()
    dev = stamps.device
    lab = torch.from_numpy(labels.astype(np.float32)).to(dev)
    rng = np.random.Generator(np.random.PCG64(seed))
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    history = []
    for ep in range(epochs):
        idx = torch.from_numpy(balanced_index(labels, rng)).to(dev)
        tot = torch.zeros(1, dtype=torch.float64, device=dev)
        steps = 0
        for b0 in range(0, idx.numel() - batch + 1, batch):
            net.train_step(stamps, lab, index=idx[b0:b0 + batch], lr=lr, loss=loss)
            tot += loss
            steps += 1
        history.append(float(tot.item()) / max(1, steps))
        if log:
            log(f"epoch {ep + 1}/{epochs}: loss {history[-1]:.4f}")
    return history


def scores(net: Net, stamps, batch: int | None = None) -> np.ndarray:
    torch = _torch()
    n = stamps.shape[0]
    batch = batch or net.max_batch
    out = torch.empty(n, dtype=torch.float32, device=stamps.device)
    for b0 in range(0, n, batch):
        nn = min(batch, n - b0)
        net.forward(stamps[b0:b0 + nn], logits=out[b0:b0 + nn])
    return out.cpu().numpy()


def operating_point(logits: np.ndarray, labels: np.ndarray, keep: float = 0.95) -> float:
    """Logit threshold that accepts the fraction `keep` of the positive examples (chosen on data
    held out from training)."""
    pos = np.sort(np.asarray(logits)[np.asarray(labels) > 0.5])
    if pos.size == 0:
        return 0.0
    return float(pos[int(np.floor((1.0 - keep) * pos.size))]) - 1e-6


def precision_recall(accept: np.ndarray, labels: np.ndarray, tone_ids: np.ndarray, tones_injected: int):
    """Precision over the accepted candidates; recall over the injected tones (a tone is
    recovered when any of its candidates is accepted)."""
    tp = float(np.sum(accept & (labels > 0.5)))
    prec = tp / max(1.0, float(np.sum(accept)))
    found = len(np.unique(tone_ids[accept & (tone_ids >= 0)]))
    return prec, found / max(1, tones_injected)
