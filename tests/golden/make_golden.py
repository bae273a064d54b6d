"""Writes oracle reference values for the named fragment workloads.

Runs only the FP64 oracle (oracle/) on the seeded synthetic inputs (synth/)
and stores energies, iteration counts, amplitude norms and a seeded sample of
amplitude elements as JSON next to this script.  A name with the suffix
":mp2" stores only the MP2 energy and the MP1 amplitudes (sample and norm), which
the oracle computes in seconds even at the large workload's full size ("batch:mp2":
each of the 64 fragments of the batched workload).  "batch:ccsd" stores
converged CCSD and (T) values for the fragments of the batched workload listed in
synth.BATCH_ORACLE_SUBSET (written after each fragment), and "large:triples" the (T)
energy at the large workload's virtual and auxiliary size with few occupied
orbitals on seeded amplitudes (synth.LARGE_TRIPLES_SHAPE).  Usage:

    python tests/golden/make_golden.py single_small single_realistic large:mp2 batch:mp2 \
        batch:ccsd large:triples
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ccsd as occ, triples as otr  # noqa: E402
from synth import (BATCH_ORACLE_SUBSET, CONFIG_SHAPES, LARGE_TRIPLES_SHAPE,  # noqa: E402
                   batch_shapes, make_fragment, random_amplitudes)

CONV_TOL = 1e-10
NSAMPLE = 256


def golden(name: str) -> dict:
    o, v, X, seed = CONFIG_SHAPES[name]
    return solve_and_sample(name, o, v, X, seed)


def solve_and_sample(name: str, o: int, v: int, X: int, seed: int) -> dict:
    """Converged oracle CCSD and (T) of one synthetic fragment, with samples."""
    f = make_fragment(o, v, X, seed)
    t0 = time.time()
    r = occ.ccsd(f.B, f.eps_occ, f.eps_vir, conv_tol=CONV_TOL, max_iter=200)
    t_cc = time.time() - t0
    t0 = time.time()
    e_t = otr.e_triples_restricted(f.B, f.eps_occ, f.eps_vir, r.t1, r.t2)
    t_t = time.time() - t0
    rng = np.random.default_rng(12345)
    idx2 = np.stack([rng.integers(0, o, NSAMPLE), rng.integers(0, o, NSAMPLE),
                     rng.integers(0, v, NSAMPLE), rng.integers(0, v, NSAMPLE)], axis=1)
    idx1 = np.stack([rng.integers(0, o, 64), rng.integers(0, v, 64)], axis=1)
    return {
        "workload": name, "nocc": o, "nvir": v, "naux": X, "seed": seed,
        "input_sha256": f.sha256(), "conv_tol": CONV_TOL,
        "converged": bool(r.converged), "n_iter": int(r.n_iter), "residual": r.residual,
        "e_mp2": r.e_mp2, "e_ccsd": r.e_ccsd, "e_t": e_t,
        "t1_norm": float(np.linalg.norm(r.t1)), "t2_norm": float(np.linalg.norm(r.t2)),
        "t2_index": idx2.tolist(), "t2_value": [float(r.t2[tuple(i)]) for i in idx2],
        "t1_index": idx1.tolist(), "t1_value": [float(r.t1[tuple(i)]) for i in idx1],
        "oracle_seconds": {"ccsd": t_cc, "triples": t_t},
    }


def golden_mp2(name: str) -> dict:
    """MP1 amplitudes (Eq. 21 with every occupied orbital) and the MP2 energy
    (Eq. 7 at T1 = 0) of one workload."""
    o, v, X, seed = CONFIG_SHAPES[name]
    f = make_fragment(o, v, X, seed)
    t0 = time.time()
    t2, e_mp2 = occ.mp2(f.B, f.eps_occ, f.eps_vir)
    t_mp2 = time.time() - t0
    rng = np.random.default_rng(12345)
    idx2 = np.stack([rng.integers(0, o, NSAMPLE), rng.integers(0, o, NSAMPLE),
                     rng.integers(0, v, NSAMPLE), rng.integers(0, v, NSAMPLE)], axis=1)
    return {
        "workload": name, "nocc": o, "nvir": v, "naux": X, "seed": seed,
        "input_sha256": f.sha256(), "e_mp2": e_mp2,
        "t2_norm": float(np.linalg.norm(t2)),
        "t2_index": idx2.tolist(), "t2_value": [float(t2[tuple(i)]) for i in idx2],
        "oracle_seconds": {"mp2": t_mp2},
    }


def golden_batch_mp2() -> dict:
    """Per-fragment MP2 energy, MP1 amplitude norm and 8 sampled MP1 amplitudes of
    the 64 fragments of the batched workload."""
    rng = np.random.default_rng(54321)
    out = []
    t0 = time.time()
    for (o, v, X, seed) in batch_shapes():
        f = make_fragment(o, v, X, seed)
        t2, e_mp2 = occ.mp2(f.B, f.eps_occ, f.eps_vir)
        idx2 = np.stack([rng.integers(0, o, 8), rng.integers(0, o, 8),
                         rng.integers(0, v, 8), rng.integers(0, v, 8)], axis=1)
        out.append({"shape": [o, v, X, seed], "input_sha256": f.sha256(), "e_mp2": e_mp2,
                    "t2_norm": float(np.linalg.norm(t2)), "t2_index": idx2.tolist(),
                    "t2_value": [float(t2[tuple(i)]) for i in idx2]})
    return {"workload": "batch", "fragments": out, "e_mp2": sum(x["e_mp2"] for x in out),
            "oracle_seconds": {"mp2": time.time() - t0}}


def golden_batch_ccsd(path: str) -> dict:
    """Converged CCSD and (T) of the subset of batched-workload fragments; the
    file is rewritten after each fragment (smallest first)."""
    shapes = batch_shapes()
    subset = sorted(BATCH_ORACLE_SUBSET,
                    key=lambda k: shapes[k][0] ** 3 * shapes[k][1] ** 4)
    out = {"workload": "batch", "subset": list(subset), "fragments": []}
    for k in subset:
        o, v, X, seed = shapes[k]
        g = solve_and_sample(f"batch[{k}]", o, v, X, seed)
        g["index"] = k
        out["fragments"].append(g)
        with open(path, "w") as fh:
            json.dump(out, fh, indent=1)
        print(f"batch[{k}] {o} {v} {X}: iters {g['n_iter']} E_CCSD {g['e_ccsd']:.12f} "
              f"E_T {g['e_t']:.12f} {g['oracle_seconds']}", flush=True)
    return out


def golden_large_triples() -> dict:
    """(T) (restricted and, as a check, nothing else) on seeded amplitudes at the
    large workload's virtual and auxiliary size."""
    o, v, X, seed, aseed = LARGE_TRIPLES_SHAPE
    f = make_fragment(o, v, X, seed)
    t1, t2 = random_amplitudes(o, v, aseed)
    t0 = time.time()
    e_t = otr.e_triples_restricted(f.B, f.eps_occ, f.eps_vir, t1, t2)
    h = __import__("hashlib").sha256()
    h.update(t1.tobytes())
    h.update(t2.tobytes())
    return {"workload": "large_triples", "nocc": o, "nvir": v, "naux": X, "seed": seed,
            "amplitude_seed": aseed, "input_sha256": f.sha256(),
            "amplitude_sha256": h.hexdigest(), "e_t": e_t,
            "oracle_seconds": {"triples": time.time() - t0}}


if __name__ == "__main__":
    for arg in sys.argv[1:] or ["single_small"]:
        name, _, part = arg.partition(":")
        here = os.path.dirname(os.path.abspath(__file__))
        if part == "ccsd" and name == "batch":
            path = os.path.join(here, "batch_ccsd.json")
            golden_batch_ccsd(path)
            continue
        if part == "triples" and name == "large":
            g = golden_large_triples()
            path = os.path.join(here, "large_triples.json")
            with open(path, "w") as fh:
                json.dump(g, fh, indent=1)
            print(arg, g["e_t"], g["oracle_seconds"], flush=True)
            continue
        if part == "mp2":
            g = golden_batch_mp2() if name == "batch" else golden_mp2(name)
            path = os.path.join(here, f"{name}_mp2.json")
        else:
            g = golden(name)
            path = os.path.join(here, f"{name}.json")
        with open(path, "w") as fh:
            json.dump(g, fh, indent=1)
        print(arg, {k: g[k] for k in ("e_mp2", "oracle_seconds")}, flush=True)
