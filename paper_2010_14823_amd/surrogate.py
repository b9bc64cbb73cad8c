"""Training driver of the process-rate surrogate (orchestration only).

Every computation -- the plain-path rate samples, the statistics, the
forward/backward passes, Adam and the bfloat16 inference -- runs in
libcasim's kernels; this module only loops over seeds, epochs and batches,
draws the seeded batch permutations (random numbers of the method are passed
in as inputs) and keeps device buffers.

Training set: points where anything can happen, sampled with equal
probability from LES-like domains (256 x 256 columns x 100 levels, 50 %
clustered cloud, dt = 2 s) of seeds 10..19, ~400,000 per seed; a random 10 %
of the samples (seeded) is held out for validation, and the parameters of
the epoch with the lowest validation loss are kept.
"""
from __future__ import annotations

import time

import numpy as np

from . import casim, synth


def training_config(seed: int) -> synth.Config:
    return synth.Config("train_s%d" % seed, 256, 256, 100, seed, 0.5)


def generate_samples(seeds=range(10, 20), per_seed=400_000, dt=2.0, log=print):
    """Plain-path samples from several seeded domains, concatenated on the device.

    Returns dict(feat, rates, gates, n, val_mask) with torch tensors on cuda.
    """
    import torch
    seeds = list(seeds)
    cap = per_seed * len(seeds)
    feat = torch.empty((cap, 12), dtype=torch.float32, device="cuda")
    rates = torch.empty((cap, 12), dtype=torch.float32, device="cuda")
    gates = torch.empty((cap,), dtype=torch.int16, device="cuda")
    n = 0
    for s in seeds:
        cfg = training_config(s)
        st_h, dz = synth.generate_stacked(cfg, workers=8)
        st = torch.from_numpy(st_h).cuda()
        del st_h
        tend = torch.empty((12, cfg.nlev, cfg.ncol), dtype=torch.float64, device="cuda")
        sfc = torch.empty((8, cfg.ncol), dtype=torch.float64, device="cuda")
        # keep probability so that about per_seed of the active points are sampled
        _, n_active = casim.rates_dump(st, dz, cfg.dt, s, 1.0, 0, None, None, None, tend, sfc)
        keep = min(1.0, per_seed / max(1, n_active))
        got, _ = casim.rates_dump(st, dz, cfg.dt, s, keep, min(per_seed, cap - n), feat[n:], rates[n:],
                                  gates[n:], tend, sfc)
        n += got
        log("surrogate: seed %d -> %d samples (keep %.4f)" % (s, got, keep))
        del st, tend, sfc
    is_val = np.random.default_rng(12345).uniform(size=n) < 0.1
    return {"feat": feat, "rates": rates, "gates": gates, "n": n, "is_val": is_val}


class Trainer:
    """Adam training of the surrogate on prepared device tensors."""

    def __init__(self, data, seed=0, log=print):
        import torch
        self.log = log
        self.n = data["n"]
        n = self.n
        self.x = torch.empty((n, 12), dtype=torch.float32, device="cuda")
        self.y = torch.empty_like(self.x)
        self.m = torch.empty_like(self.x)
        self.stats = casim.mlp_fit_stats(data["feat"], data["rates"], data["gates"], n)
        casim.mlp_prepare(data["feat"], data["rates"], data["gates"], n, self.x, self.y, self.m)
        self.train_idx = np.nonzero(~data["is_val"])[0].astype(np.int32)
        self.val_idx = np.nonzero(data["is_val"])[0].astype(np.int32)
        self.rng = np.random.default_rng(seed)
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        self.grad = torch.empty(casim.MLP_NPARAMS, dtype=torch.float32, device="cuda")
        casim.mlp_init(seed)

    def eval_loss(self, idx) -> float:
        import torch
        dev = torch.from_numpy(idx).cuda()
        tot, w = 0.0, 0
        for o in range(0, len(idx), casim.MLP_MAX_BATCH):
            b = min(casim.MLP_MAX_BATCH, len(idx) - o)
            casim.mlp_grad(self.x, self.y, self.m, dev[o:], b, self.grad, self.loss)
            tot += float(self.loss.item()) * b
            w += b
        return tot / max(1, w)

    def fit(self, epochs=10, batch=4096, lr=2e-3, lr_final=1e-4):
        import torch
        hist = []
        best, best_blob = float("inf"), None
        steps_per_epoch = len(self.train_idx) // batch
        total = epochs * steps_per_epoch
        step = 0
        for ep in range(epochs):
            t0 = time.perf_counter()
            perm = self.train_idx[self.rng.permutation(len(self.train_idx))]
            dev = torch.from_numpy(perm).cuda()
            for b in range(steps_per_epoch):
                # cosine decay from lr to lr_final
                frac = step / max(1, total - 1)
                cur = lr_final + 0.5 * (lr - lr_final) * (1.0 + np.cos(np.pi * frac))
                casim.mlp_train_step(self.x, self.y, self.m, dev[b * batch:], batch, cur, self.loss)
                step += 1
            torch.cuda.synchronize()
            tl = float(self.loss.item())
            vl = self.eval_loss(self.val_idx)
            hist.append({"epoch": ep, "train_batch_loss": tl, "val_loss": vl,
                         "seconds": time.perf_counter() - t0})
            self.log("surrogate: epoch %d train %.4f val %.4f (%.1f s)" % (ep, tl, vl, hist[-1]["seconds"]))
            if vl < best:
                best, best_blob = vl, casim.mlp_save()
        if best_blob is not None:
            casim.mlp_load(best_blob)
        self.best_val = best
        return hist


def main(argv=None):
    """python -m paper_2010_14823_amd.surrogate --out CKPT [--epochs E] ..."""
    import argparse
    import json
    ap = argparse.ArgumentParser(description="train the process-rate surrogate on plain-path samples")
    ap.add_argument("--out", required=True, help="checkpoint file to write")
    ap.add_argument("--seeds", default="10-19")
    ap.add_argument("--per-seed", type=int, default=400_000)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    a = ap.parse_args(argv)
    lo, hi = (int(x) for x in a.seeds.split("-"))
    casim.init()
    t0 = time.perf_counter()
    data = generate_samples(range(lo, hi + 1), a.per_seed, log=lambda m: print(m, flush=True))
    t1 = time.perf_counter()
    tr = Trainer(data, seed=a.seed, log=lambda m: print(m, flush=True))
    untrained = tr.eval_loss(tr.val_idx)
    hist = tr.fit(epochs=a.epochs, batch=a.batch, lr=a.lr)
    t2 = time.perf_counter()
    blob = casim.mlp_save()
    with open(a.out, "wb") as f:
        f.write(blob)
    print(json.dumps({"samples": data["n"], "train": len(tr.train_idx), "val": len(tr.val_idx),
                      "untrained_val_loss": untrained, "best_val_loss": tr.best_val, "history": hist,
                      "sample_seconds": t1 - t0, "train_seconds": t2 - t1}), flush=True)


if __name__ == "__main__":
    main()
