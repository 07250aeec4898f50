"""Learned per-vector filter degree: traces from the solver, labels, training on the GPU with the
library's own forward/backward/Adam kernels, and the weights blob for chfsi_set_degree_model.

The paper filters every vector with one fixed degree (Section 3.1; Table 3: 25) and notes that the
degree barely matters once it is high enough.  Here a 5 -> 64 -> 64 -> 64 -> 1 network predicts a
degree per vector from
  t = (theta - c)/e       where the Ritz value sits relative to the damped interval [a, b],
  log10(r / tau)          its residual relative to the locking threshold,
  (a - mu1)/(b - mu1)     and (b - mu1)/(|mu1| + |b|), the shape of the filter interval,
  d_prev                  the degree it was filtered with in the loop that produced (theta, r).
Label of a traced vector: the degree that would have brought its residual from r to tau in one
loop at the contraction per step observed in the trace, kappa = (r_after / r) ** (1 / d):
  d* = ceil(ln(r / tau) / -ln kappa), clamped to [dmin, dmax] (dmax if kappa >= 1).
Traces come from solves whose degrees are drawn uniformly in [dmin, dmax] (CHFSI_DEG_RANDOM).
At inference the predicted degree is raised by a margin (chfsi_params.deg_margin, LEARNED_MARGIN
below): an underestimated degree costs a whole extra loop of the block (QR, Rayleigh-Ritz), a
slightly high one a few matrix-vector products.
"""
from __future__ import annotations

import json
import math
import os
from typing import Iterable, List, Optional, Tuple

import numpy as np

from . import chfsi, synth

NF = 5
NPARAM = chfsi.MLP_NPARAM
MODEL_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "degree_model.npy")
META_PATH = os.path.splitext(MODEL_PATH)[0] + "_meta.json"
TRAIN_SEEDS = tuple(range(1, 9))   # traces of the n = 4096 sequence
SELECT_SEED = 9                    # margin and best fixed degree are chosen on this sequence
EVAL_SEED = 0                      # held out: used only to report
MARGINS = (0, 1, 2, 3, 4)
FIXED_DEGREES = (8, 12, 16, 20, 25)


def meta(path: str = META_PATH) -> dict:
    """Provenance of the committed network: training seeds and cycles, the margin and the best
    fixed degree chosen on the selection seed (never on the evaluation seed)."""
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


LEARNED_MARGIN = int(meta().get("margin", 2))   # degree margin of the learned policy


def features(tr: np.ndarray) -> np.ndarray:
    """Trace rows -> network features (N x 5, float64)."""
    f = np.empty((tr.shape[0], NF))
    f[:, 0] = tr[:, 2]
    f[:, 1] = tr[:, 3] - np.log10(tr[:, 9])
    f[:, 2] = tr[:, 4]
    f[:, 3] = tr[:, 5]
    f[:, 4] = tr[:, 6]
    return f


def labels(tr: np.ndarray, dmin: int = 4, dmax: int = 30) -> Tuple[np.ndarray, np.ndarray]:
    """(labels, valid mask) from the contraction observed between a row and the next loop."""
    r = 10.0 ** tr[:, 3]
    r_after = tr[:, 8]
    d = tr[:, 7]
    thr = tr[:, 9]
    valid = (r_after > 0) & np.isfinite(r_after) & (d > 0)
    lab = np.full(tr.shape[0], float(dmax))
    done = valid & (r <= thr)
    lab[done] = dmin
    live = valid & (r > thr)
    with np.errstate(divide="ignore", invalid="ignore"):
        kappa = (r_after[live] / r[live]) ** (1.0 / d[live])
        need = np.log(r[live] / thr[live])
        est = np.where(kappa < 1.0, np.ceil(need / -np.log(np.maximum(kappa, 1e-300))), dmax)
    lab[live] = np.clip(est, dmin, dmax)
    return lab, valid


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights, zero biases, output bias so that the initial degree is mid-range."""
    rng = np.random.default_rng(seed)
    P = np.zeros(NPARAM, dtype=np.float32)
    o = 0
    for nin, nout in ((NF, 64), (64, 64), (64, 64), (64, 1)):
        P[o:o + nin * nout] = rng.standard_normal(nin * nout) * math.sqrt(2.0 / nin)
        o += nin * nout + nout
    return P


def generate_traces(h: chfsi.Handle, spec: synth.SequenceSpec, dmin: int = 4, dmax: int = 30,
                    seed_offset: int = 0) -> np.ndarray:
    """Solves every cycle of spec (warm-started) with random per-vector degrees; returns all trace
    rows (CHFSI_TRACE_COLS columns)."""
    from . import sequence
    seq = sequence.Sequence(spec, handle=h)
    rows = []
    for c in range(spec.cycles):
        r = seq.solve(c, warm=c > 0, store=True, degree_policy=chfsi.DEG_RANDOM, trace=1, deg_min=dmin,
                      deg_max=dmax, seed=spec.seed * 1000 + c + seed_offset)
        if r.status == 0:
            rows.append(h.get_trace())
    return np.concatenate(rows) if rows else np.zeros((0, chfsi.TRACE_COLS))


def train(h: chfsi.Handle, X: np.ndarray, y: np.ndarray, epochs: int = 40, batch: int = 256, lr: float = 1e-3,
          seed: int = 0, dmin: float = 4.0, dmax: float = 30.0):
    """Normalises the features and trains the network on the GPU (chfsi_mlp_train).  Returns
    (params float32, mean, std, per-epoch loss)."""
    import torch
    mean = X.mean(axis=0)
    std = X.std(axis=0)
    std[std < 1e-6] = 1.0
    Xn = ((X - mean) / std).astype(np.float32)
    dev = f"cuda:{h.device}"
    dP = torch.from_numpy(init_params(seed)).to(dev)
    dX = torch.from_numpy(np.ascontiguousarray(Xn)).to(dev)
    dy = torch.from_numpy(y.astype(np.float32)).to(dev)
    hist = h.mlp_train(dP, dX, dy, epochs=epochs, batch=batch, lr=lr, seed=seed, dmin=dmin, dmax=dmax)
    return dP.cpu().numpy(), mean.astype(np.float32), std.astype(np.float32), hist


def make_blob(P: np.ndarray, mean: np.ndarray, std: np.ndarray) -> np.ndarray:
    return np.concatenate([P.astype(np.float32), mean.astype(np.float32), std.astype(np.float32)])


def save(blob: np.ndarray, path: str = MODEL_PATH) -> None:
    np.save(path, blob.astype(np.float32))


def load(path: str = MODEL_PATH) -> Optional[np.ndarray]:
    return np.load(path) if os.path.exists(path) else None


def run_policy(h: chfsi.Handle, seq, policy: int, deg: int = 12, precision: int = 0,
               cycles: Optional[int] = None, margin: Optional[int] = None) -> dict:
    """Solves the (device-resident) sequence warm-started with one degree policy; totals of time,
    matvecs and loops over the warm cycles 1 .. (cycle 0 starts from a random block and is the
    same for every policy).  The stored solutions of a previous run are discarded first.  margin:
    deg_margin (default LEARNED_MARGIN for the learned policy, 0 otherwise)."""
    if margin is None:
        margin = LEARNED_MARGIN if policy == chfsi.DEG_LEARNED else 0
    spec = seq.spec
    ncyc = cycles or spec.cycles
    seq.X = [None] * spec.cycles
    seq.lam = [None] * spec.cycles
    tot = dict(ms=0.0, matvecs=0, loops=0, filter_ms=0.0, ok=True, max_resid=0.0, lam=[])
    for c in range(ncyc):
        r = seq.solve(c, warm=c > 0, store=True, degree_policy=policy, deg=deg, filter_precision=precision,
                      deg_margin=margin)
        tot["ok"] &= r.status == 0
        if c == 0:
            continue
        tot["ms"] += r.wall_ms
        tot["matvecs"] += r.stats["matvecs"]
        tot["loops"] += r.stats["loops"]
        tot["filter_ms"] += r.stats["t_filter"]
        tot["max_resid"] = max(tot["max_resid"], float(r.resid[:spec.nev].max()))
        tot["lam"].append(r.lam[:spec.nev].copy())
    return tot


def _summary(v: dict) -> dict:
    out = {q: (round(v[q], 1) if isinstance(v[q], float) else v[q]) for q in ("ms", "matvecs", "loops", "filter_ms", "ok")}
    out["max_resid"] = float(v["max_resid"])
    return out


def main(argv: Iterable[str] = ()) -> int:
    """Traces of the training seeds (20-cycle n=4096 sequences, random per-vector degrees), training
    on the GPU, then on the selection seed: the learned policy's margin and the analytic rule's
    (from MARGINS) and the best fixed degree (from FIXED_DEGREES), by time to solution over the
    warm cycles.  Writes the blob and its provenance (META_PATH); the evaluation seed is not touched
    here.  --select-only repeats the selection with the saved network."""
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--cycles", type=int, default=20, help="cycles of every sequence")
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--out", default=MODEL_PATH)
    ap.add_argument("--select-only", action="store_true")
    a = ap.parse_args(list(argv))
    import torch
    from . import sequence
    h = chfsi.Handle(0)
    if a.select_only:
        blob = load(a.out)
        info = meta(os.path.splitext(a.out)[0] + "_meta.json")
        return _select(h, a, blob, info)
    trs = []
    for s in TRAIN_SEEDS:
        spec = synth.config_learned_degree(seed=s, n=a.n, cycles=a.cycles)
        trs.append(generate_traces(h, spec))
        print(json.dumps({"seed": s, "rows": int(trs[-1].shape[0])}), flush=True)
        torch.cuda.empty_cache()
    tr = np.concatenate(trs)
    y, valid = labels(tr)
    X = features(tr)[valid]
    y = y[valid]
    P, mean, std, hist = train(h, X, y, epochs=a.epochs)
    print(json.dumps({"samples": int(len(y)), "loss_first": float(hist[0]), "loss_last": float(hist[-1])}), flush=True)
    blob = make_blob(P, mean, std)
    save(blob, a.out)
    np.save(os.path.splitext(a.out)[0] + "_loss.npy", np.asarray(hist))
    info = {"n": a.n, "cycles": a.cycles, "train_seeds": list(TRAIN_SEEDS), "samples": int(len(y)),
            "epochs": a.epochs, "loss_first": float(hist[0]), "loss_last": float(hist[-1])}
    return _select(h, a, blob, info)


def _select(h: chfsi.Handle, a, blob: np.ndarray, info: dict) -> int:
    """The selection on SELECT_SEED: margins of the learned policy and of the analytic rule, best
    fixed degree; written into the network's provenance file."""
    from . import sequence
    h.set_degree_model(blob)
    seqv = sequence.Sequence(synth.config_learned_degree(seed=SELECT_SEED, n=a.n, cycles=a.cycles), handle=h)
    sel = {}
    for mg in MARGINS:
        sel[f"learned+{mg}"] = run_policy(h, seqv, chfsi.DEG_LEARNED, margin=mg)
    for mg in MARGINS:
        sel[f"analytic+{mg}"] = run_policy(h, seqv, chfsi.DEG_ANALYTIC, margin=mg)
    for d in FIXED_DEGREES:
        sel[f"fixed{d}"] = run_policy(h, seqv, chfsi.DEG_FIXED, deg=d)
    h.set_degree_model(None)
    for k, v in sel.items():
        print(json.dumps({"selection": k, **_summary(v)}), flush=True)
    pick = lambda keys: min((k for k in keys if sel[k]["ok"]), key=lambda k: sel[k]["ms"])   # noqa: E731
    margin = int(pick([f"learned+{mg}" for mg in MARGINS]).split("+")[1])
    margin_an = int(pick([f"analytic+{mg}" for mg in MARGINS]).split("+")[1])
    best_fixed = int(pick([f"fixed{d}" for d in FIXED_DEGREES])[5:])
    info.update({"selection_seed": SELECT_SEED, "margin": margin, "analytic_margin": margin_an,
                 "best_fixed_degree": best_fixed, "selection": {k: _summary(v) for k, v in sel.items()}})
    with open(os.path.splitext(a.out)[0] + "_meta.json", "w") as fh:
        json.dump(info, fh, indent=1)
    print(json.dumps({"margin": margin, "analytic_margin": margin_an, "best_fixed_degree": best_fixed}), flush=True)
    return 0


if __name__ == "__main__":
    import sys
    sys.exit(main(sys.argv[1:]))
