"""Training driver of the learned T2 starting guess (argument marshalling and
bookkeeping only: features, network, loss, gradients and Adam run in the
library's kernels through the lnocc_mlp_* calls).

    python -m paper_2407_11258_amd.learned --train 64 --eval 16 --out model.pt
    python -m paper_2407_11258_amd.learned --load model.pt --eval 512

solves `train` synthetic fragments of the realistic shape (nocc=16, nvir=160,
naux=528; seeds 100000 + k), samples amplitudes of each converged T2 as
(features, t_CCSD - t_MP1) pairs, trains the network (or loads one with
--load), then solves `eval` held-out fragments (seeds 200000 + k) from the MP2
start and from the learned start and prints one JSON line: iterations, times
and energy differences.  Fragments are generated on the host in a thread pool
ahead of the device work.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import sys
import time

import numpy as np

from . import lnocc as L

F = L.LNOCC_MLP_FEATURES


def _torch():
    import torch
    return torch


def _check(st: int, what: str) -> None:
    if st < 0:
        raise RuntimeError(f"{what}: {L.lnocc_status_string(st)}: {L.lnocc_last_error()}")


class LearnedGuess:
    """A model blob and its Adam moments on the device."""

    def __init__(self, device="cuda"):
        torch = _torch()
        self.device = device
        self.blob = torch.zeros(L.LNOCC_MLP_BLOB, dtype=torch.float32, device=device)
        self.adam = torch.zeros(2 * L.LNOCC_MLP_PARAMS, dtype=torch.float32, device=device)
        self.steps = 0
        self._ws = L.Workspace(device)

    def _opt(self, rows: int, training: bool):
        st, nbytes = L.lnocc_mlp_workspace_bytes(rows, training)
        _check(st, "workspace size")
        buf = self._ws.ensure(nbytes)
        opt = L.lnocc_default_options()
        opt.workspace, opt.workspace_bytes = buf.data_ptr(), buf.numel()
        opt.stream = _torch().cuda.current_stream().cuda_stream
        return opt

    def init(self, X, Y, seed: int = 0) -> None:
        _check(L.lnocc_mlp_init(self.blob.data_ptr(), X.data_ptr(), Y.data_ptr(), Y.numel(), seed,
                                self._opt(1 << 16, False)), "init")
        self.adam.zero_()
        self.steps = 0

    def train(self, X, Y, steps: int, batch: int = 65536, lr: float = 1e-3, seed: int = 1,
              lr_final: float | None = None, log_every: int = 0) -> list:
        """Adam steps; with lr_final the rate follows a cosine from lr to lr_final
        (held constant over each chunk of 100 steps)."""
        opt = self._opt(batch, True)
        losses = []
        chunk = 100 if lr_final is not None else steps
        done = 0
        while done < steps:
            m = min(chunk, steps - done)
            rate = lr
            if lr_final is not None:
                rate = lr_final + 0.5 * (lr - lr_final) * (1 + np.cos(np.pi * done / steps))
            st, ls = L.lnocc_mlp_train(self.blob.data_ptr(), self.adam.data_ptr(), self.steps, m,
                                       X.data_ptr(), Y.data_ptr(), Y.numel(), batch, rate, seed,
                                       opt)
            _check(st, "train")
            self.steps += m
            done += m
            losses.extend(ls)
            if log_every and (done % log_every < m or done == steps):
                print(f"[learned] step {self.steps}: minibatch loss {np.mean(ls):.4e} "
                      f"(lr {rate:.2e})", file=sys.stderr, flush=True)
        return losses

    def predict(self, X):
        torch = _torch()
        out = torch.empty(X.shape[0], dtype=torch.float32, device=self.device)
        _check(L.lnocc_mlp_predict(self.blob.data_ptr(), X.data_ptr(), X.shape[0], out.data_ptr(),
                                   self._opt(1 << 16, False)), "predict")
        return out

    def loss_grad(self, X, Y):
        torch = _torch()
        grad = torch.empty(L.LNOCC_MLP_PARAMS, dtype=torch.float32, device=self.device)
        st, loss = L.lnocc_mlp_loss_grad(self.blob.data_ptr(), X.data_ptr(), Y.data_ptr(),
                                         Y.numel(), grad.data_ptr(), self._opt(Y.numel(), True))
        _check(st, "loss_grad")
        return loss, grad

    def save(self, path) -> None:
        _torch().save({"blob": self.blob.cpu(), "steps": self.steps}, path)

    def load(self, path) -> None:
        d = _torch().load(path, weights_only=True)
        self.blob.copy_(d["blob"])
        self.steps = int(d["steps"])


def fragment_tensors(frag, device="cuda"):
    torch = _torch()
    return tuple(torch.tensor(x, dtype=torch.float64, device=device)
                 for x in (frag.B, frag.eps_occ, frag.eps_vir))


def collect_samples(dev_frags, per_fragment: int, seed: int, precision: str = "fp32",
                    conv_tol: float = 1e-8, batch_slots: int = 4, batch_streams: int = 4):
    """Solve the fragments, then draw per_fragment amplitudes of each converged T2
    (uniformly, numpy generator seeded by seed + k) as feature / target rows."""
    torch = _torch()
    res = L.solve_batch(dev_frags, conv_tol=conv_tol, precision=precision, do_triples=False,
                        batch_slots=batch_slots, batch_streams=batch_streams)
    n = per_fragment * len(dev_frags)
    X = torch.empty((n, F), dtype=torch.float32, device="cuda")
    Y = torch.empty(n, dtype=torch.float32, device="cuda")
    ws = L.Workspace("cuda")
    for k, ((B, eo, ev), r) in enumerate(zip(dev_frags, res)):
        if r.status < 0:
            raise RuntimeError(f"training fragment {k}: {L.lnocc_status_string(r.status)}")
        o, v = eo.numel(), ev.numel()
        rng = np.random.default_rng(seed + k)
        idx = torch.tensor(rng.integers(0, o * o * v * v, per_fragment), dtype=torch.int64,
                           device="cuda")
        f = L.make_fragment_struct(B, eo, ev, r.t1, r.t2, conv_tol)
        opt = L.make_options()
        ws.attach([f], opt)
        sl = slice(k * per_fragment, (k + 1) * per_fragment)
        _check(L.lnocc_mlp_samples(f, opt, idx.data_ptr(), per_fragment, X[sl].data_ptr(),
                                   Y[sl].data_ptr()), "samples")
    return X, Y, res


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--train", type=int, default=64)
    ap.add_argument("--eval", type=int, default=16)
    ap.add_argument("--per-fragment", type=int, default=1 << 17)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=2e-5)
    ap.add_argument("--conv-tol", type=float, default=1e-7)
    ap.add_argument("--final-tol", type=float, default=1e-10,
                    help="both solves then continue from where they stopped to this step "
                         "tolerance; their energies there are the final energies compared")
    ap.add_argument("--shape", default="16,160,528")
    ap.add_argument("--out", default="")
    ap.add_argument("--load", default="", help="model file written by --out: skips the "
                    "training data and the training")
    args = ap.parse_args()
    torch = _torch()
    from synth import make_fragment
    o, v, X_ = (int(x) for x in args.shape.split(","))
    log = lambda m: print(f"[learned] {m}", file=sys.stderr, flush=True)   # noqa: E731
    # host-side fragment generation runs ahead of the device in a thread pool
    pool = cf.ThreadPoolExecutor(max_workers=8)

    def ahead(seeds):
        return [pool.submit(make_fragment, o, v, X_, s) for s in seeds]

    model = LearnedGuess("cuda")
    t_data = t_train = 0.0
    losses = []
    nsamples = 0
    if args.load:
        model.load(args.load)
    else:
        t0 = time.perf_counter()
        X, Y = [], []
        chunks = list(range(0, args.train, 16))   # 16 fragments resident at a time
        nxt = ahead(100000 + k for k in range(0, min(args.train, 16)))
        for c0 in chunks:
            cur = nxt
            c1 = c0 + 16
            nxt = ahead(100000 + k for k in range(c1, min(args.train, c1 + 16)))
            frags = [fragment_tensors(f.result()) for f in cur]
            x, y, _ = collect_samples(frags, args.per_fragment, seed=300000 + c0)
            X.append(x)
            Y.append(y)
            log(f"training data: {min(args.train, c1)}/{args.train} fragments")
            del frags
        X, Y = torch.cat(X), torch.cat(Y)
        nsamples = int(Y.numel())
        t_data = time.perf_counter() - t0
        model.init(X, Y, seed=0)
        t0 = time.perf_counter()
        losses = model.train(X, Y, args.steps, batch=args.batch, lr=args.lr,
                             lr_final=args.lr_final, log_every=500)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        del X, Y
    if args.out:
        model.save(args.out)

    rows = []
    window = 8   # held-out fragments generated ahead (about 130 MB of host memory each)
    held = ahead(200000 + k for k in range(min(window, args.eval)))
    for k in range(args.eval):
        d = fragment_tensors(held.pop(0).result())
        if k + window < args.eval:
            held += ahead([200000 + k + window])
        out = {}
        for name, kw in (("mp2", {}), ("mlp", {"guess": L.LNOCC_GUESS_MLP, "mlp": model.blob})):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            r = L.solve(*d, conv_tol=args.conv_tol, do_triples=False, **kw)
            torch.cuda.synchronize()
            out[name] = (r, time.perf_counter() - t1)
        (a, ta), (b, tb) = out["mp2"], out["mlp"]
        fin = [L.solve(*d, conv_tol=args.final_tol, do_triples=False, t1=x.t1, t2=x.t2,
                       guess=L.LNOCC_GUESS_USER) for x in (a, b)]
        rows.append({"seed": 200000 + k, "iters_mp2": a.n_iter, "iters_mlp": b.n_iter,
                     "s_mp2": ta, "s_mlp": tb, "guess_used": b.guess_used,
                     "d_e_ccsd": b.e_ccsd - a.e_ccsd,
                     "d_e_ccsd_final": fin[1].e_ccsd - fin[0].e_ccsd,
                     "status": [a.status, b.status, fin[0].status, fin[1].status]})
        log(f"held-out {k}: iterations {a.n_iter} (MP2 start) vs {b.n_iter} (learned), "
            f"dE {b.e_ccsd - a.e_ccsd:.1e}, final dE {fin[1].e_ccsd - fin[0].e_ccsd:.1e}")
    pool.shutdown()
    mean = lambda key: float(np.mean([r[key] for r in rows])) if rows else None   # noqa: E731
    summary = {
        "shape": [o, v, X_], "conv_tol": args.conv_tol,
        "train_fragments": 0 if args.load else args.train, "model": args.load or None,
        "eval_fragments": args.eval,
        "samples": nsamples, "steps": 0 if args.load else args.steps, "batch": args.batch,
        "data_seconds": t_data, "train_seconds": t_train,
        "loss_first": losses[0] if losses else None,
        "loss_last": float(np.mean(losses[-50:])) if losses else None,
        "mean_iters_mp2": mean("iters_mp2"), "mean_iters_mlp": mean("iters_mlp"),
        "mean_seconds_mp2": mean("s_mp2"), "mean_seconds_mlp": mean("s_mlp"),
        "max_abs_d_e_ccsd": float(max(abs(r["d_e_ccsd"]) for r in rows)) if rows else None,
        "final_tol": args.final_tol,
        "max_abs_d_e_ccsd_final": (float(max(abs(r["d_e_ccsd_final"]) for r in rows))
                                   if rows else None),
        "fallbacks": int(sum(r["guess_used"] != L.LNOCC_GUESS_MLP for r in rows)),
        "rows": rows,
    }
    print(json.dumps(summary), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
