"""The learned low-fidelity level: a permutation-invariant set network over
the bubbles of a cloud, trained on QoIs that the solver itself produced, and
used as the cheapest level of OF-MLMC (its coefficient alpha absorbs its
error; the solver levels remain the reference that bounds it).

Everything numeric runs in the library's kernels (ofm_nn_*): per-bubble
features, the fused phi + pool forward on BF16 matrix cores, the backward
GEMMs and the Adam step.  This module only batches sets, shuffles them on
the host and keeps the best parameters on validation loss.

Outputs (physical units): p_max, the argmax position (x, y, z) and the time
of the maximum; the loss is the library's mean squared standardised error
over the five.  The standardisation is chosen here so that the loss follows
what the control variate needs:
  * centre and spread of each output are its median and 1.4826 x median
    absolute deviation over the training set (robust to the heavy tails of
    the argmax position and time, e.g. a maximum taken at t = 0);
  * training targets are clipped to centre +- 5 spreads;
  * the spreads of the four auxiliary outputs (position, time) are widened by
    `aux_scale`, which weights their squared errors by 1 / aux_scale^2
    against p_max.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import capi

OUTPUTS = ("p_max", "x", "y", "z", "t_at_max")


def targets(qois: list) -> np.ndarray:
    """Five targets per solved sample (ofm_qoi dicts)."""
    return np.array([[q["p_max"], q["x"][0], q["x"][1], q["x"][2], q["t_at_max"]] for q in qois], dtype=np.float64)


class Surrogate:
    def __init__(self, ctx: capi.Context, cloud: dict, seed: int = 0, lr: float = 3e-3):
        self.ctx, self.cloud, self.seed, self.lr = ctx, cloud, seed, lr
        self.net = None
        self.info = {}

    # -- inputs ---------------------------------------------------------------
    def features(self, bubbles: list):
        """Device tensors: per-bubble inputs [rows, 4] float and set offsets
        [n_sets + 1] int32."""
        import torch
        sizes = [len(b) for b in bubbles]
        b = torch.tensor(np.concatenate(bubbles), dtype=torch.float64, device="cuda")
        x = torch.empty((b.shape[0], 4), dtype=torch.float32, device="cuda")
        capi.ofm_nn_features(self.cloud, b, x)
        off = torch.tensor(np.concatenate([[0], np.cumsum(sizes)]), dtype=torch.int32, device="cuda")
        return x, off

    # -- training ---------------------------------------------------------------
    def fit(self, bubbles: list, qois: list, epochs: int = 300, batch: int = 256, val_frac: float = 0.1,
            patience: int = 40, aux_scale: float = 3.0, log=print) -> dict:
        """Adam on mini-batches of sets; the parameters of the epoch with the
        best validation correlation of p_max are kept (early stopping after
        `patience` epochs without improvement)."""
        import torch
        ok = [i for i, q in enumerate(qois) if q["status"] == capi.SAMPLE_OK]
        Y = targets([qois[i] for i in ok])
        B = [np.asarray(bubbles[i], dtype=np.float64) for i in ok]
        n = len(ok)
        rng = np.random.default_rng(self.seed)
        perm = rng.permutation(n)
        n_val = max(1, int(round(val_frac * n)))
        val, tr = perm[:n_val], perm[n_val:]
        mean = np.median(Y[tr], axis=0)
        std = 1.4826 * np.median(np.abs(Y[tr] - mean), axis=0)
        fallback = Y[tr].std(axis=0)
        std = np.where(std > 0, std, np.where(fallback > 0, fallback, 1.0))
        std[1:] *= aux_scale
        Yc = np.clip(Y, mean - 5 * std, mean + 5 * std)
        self.net = capi.SetNet(self.ctx, 1.0 / float(self.cloud["n_bubbles"]), seed=self.seed, lr=self.lr,
                               out_mean=tuple(float(v) for v in mean), out_std=tuple(float(v) for v in std))
        # per-set inputs once on the device, then on the host for shuffling
        x_all, off_all = self.features(B)
        x_host = x_all.cpu().numpy()
        off_host = off_all.cpu().numpy().astype(np.int64)

        def gather(idx):
            rows = np.concatenate([np.arange(off_host[i], off_host[i + 1]) for i in idx])
            sizes = off_host[np.asarray(idx) + 1] - off_host[np.asarray(idx)]
            xo = torch.tensor(x_host[rows], device="cuda")
            oo = torch.tensor(np.concatenate([[0], np.cumsum(sizes)]), dtype=torch.int32, device="cuda")
            yo = torch.tensor(Yc[idx], dtype=torch.float32, device="cuda")
            return xo, oo, yo

        xv, ov, yv = gather(val)
        yval = Y[val, 0]
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        vloss = torch.zeros(1, dtype=torch.float32, device="cuda")
        ypred = torch.empty((len(val), 5), dtype=torch.float32, device="cuda")
        best = (-math.inf, -1)
        best_params = torch.empty(capi.SetNet.param_count(), dtype=torch.float32, device="cuda")
        hist = []
        t0 = time.perf_counter()
        for ep in range(epochs):
            order = rng.permutation(tr)
            tl, nb = 0.0, 0
            for s in range(0, len(order), batch):
                xb, ob, yb = gather(order[s:s + batch])
                self.net.train_step(xb, ob, yb, loss)
                tl += loss.item()
                nb += 1
            self.net.grads(xv, ov, yv, None, vloss)
            self.net.forward(xv, ov, ypred)
            pv = ypred[:, 0].cpu().numpy().astype(np.float64)
            corr = float(np.corrcoef(pv, yval)[0, 1]) if np.std(pv) > 0 else 0.0
            v = vloss.item()
            hist.append((tl / max(nb, 1), v, corr))
            if corr > best[0]:
                best = (corr, ep)
                self.net.get_params(best_params)
            if ep - best[1] >= patience:
                break
            if ep % 25 == 0:
                log("    epoch %d: train %.4f  validation %.4f  p_max correlation %.3f" % (
                    ep, tl / max(nb, 1), v, corr))
        self.net.set_params(best_params)
        torch.cuda.synchronize()
        self.info = dict(n_train=len(tr), n_val=len(val), epochs=len(hist), best_epoch=best[1],
                         val_corr_pmax=best[0], val_loss=hist[best[1]][1], train_loss=hist[best[1]][0],
                         seconds=time.perf_counter() - t0, out_mean=mean.tolist(), out_std=std.tolist(),
                         aux_scale=aux_scale)
        return self.info

    # -- inference ----------------------------------------------------------------
    def predict(self, bubbles: list, chunk: int = 16384) -> np.ndarray:
        """[n_sets, 5] predictions in physical units (float32 network)."""
        import torch
        out = []
        for s in range(0, len(bubbles), chunk):
            x, off = self.features(bubbles[s:s + chunk])
            y = torch.empty((off.numel() - 1, 5), dtype=torch.float32, device="cuda")
            self.net.forward(x, off, y)
            out.append(y.cpu().numpy().astype(np.float64))
        return np.concatenate(out) if out else np.zeros((0, 5))
