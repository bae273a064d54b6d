"""Writes oracle reference values for the named fragment workloads.

Runs only the FP64 oracle (oracle/) on the seeded synthetic inputs (synth/)
and stores energies, iteration counts, amplitude norms and a seeded sample of
amplitude elements as JSON next to this script.  A name with the suffix
":mp2" stores only the MP2 energy and the MP1 amplitudes (sample and norm), which
the oracle computes in seconds even at the large workload's full size ("batch:mp2":
each of the 64 fragments of the batched workload).  Usage:

    python tests/golden/make_golden.py single_small single_realistic large:mp2 batch:mp2
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
from synth import CONFIG_SHAPES, batch_shapes, make_fragment  # noqa: E402

CONV_TOL = 1e-10
NSAMPLE = 256


def golden(name: str) -> dict:
    o, v, X, seed = CONFIG_SHAPES[name]
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


if __name__ == "__main__":
    for arg in sys.argv[1:] or ["single_small"]:
        name, _, part = arg.partition(":")
        here = os.path.dirname(os.path.abspath(__file__))
        if part == "mp2":
            g = golden_batch_mp2() if name == "batch" else golden_mp2(name)
            path = os.path.join(here, f"{name}_mp2.json")
        else:
            g = golden(name)
            path = os.path.join(here, f"{name}.json")
        with open(path, "w") as fh:
            json.dump(g, fh, indent=1)
        print(arg, {k: g[k] for k in ("e_mp2", "oracle_seconds")}, flush=True)
