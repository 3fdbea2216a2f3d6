"""FP64 oracle reference for the reduced-precision form at the MovieLens-20M shape.

Writes tests/golden/c3_ml20m_holdout_ref.json from the oracle only (calls
oracle/ and synth/, nothing else).  For n_f = 64 and 128: the ML-20M-shaped
matrix (seed 1) with a seeded 1% of its ratings held out (seed 3), the shared
starting point x0 (the seeded U0, M0 rounded to FP32), then
  * ALS (Algorithm 1): f after each of the first K sweeps;
  * ALS-NCG (Algorithm 2, line search of Section V-C): f after each of the
    first K iterations, the accepted trial counts, 16 sampled rows of U and of
    M after K iterations and the RMSE of u_i . m_j on the held-out ratings.
These are the FP64 values the reduced-precision runs are reported against.

Usage: python tests/golden/make_c3_ref.py [--threads 4] [--iters 3]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "c3_ml20m_holdout_ref.json")
HOLDOUT_FRAC, HOLDOUT_SEED, SAMPLE_SEED, N_SAMPLE = 0.01, 3, 5, 16


def sample_rows(n_u, n_m):
    rng = np.random.default_rng(SAMPLE_SEED)
    return (np.sort(rng.choice(n_u, N_SAMPLE, replace=False)),
            np.sort(rng.choice(n_m, N_SAMPLE, replace=False)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--iters", type=int, default=3)
    ap.add_argument("--nf", type=int, nargs="*", default=[64, 128])
    args = ap.parse_args()
    threads = oracle.set_threads(args.threads)
    out = {"citation": "Eq. (1) loss, Algorithm 1 (ALS) and Algorithm 2 (ALS-NCG, Eq. (8), "
                       "line search of Section V-C) in FP64 on the held-out-split matrix",
           "written_by": "tests/golden/make_c3_ref.py (FP64 oracle only)",
           "holdout": {"frac": HOLDOUT_FRAC, "seed": HOLDOUT_SEED},
           "sample": {"seed": SAMPLE_SEED, "n": N_SAMPLE}, "threads": threads, "configs": {}}
    for n_f in args.nf:
        t0 = time.time()
        P = synth.c1_ml20m(n_f=n_f)
        Ptr, held = synth.holdout_split(P, HOLDOUT_FRAC, HOLDOUT_SEED)
        hr, hc, hv = held
        U0 = P.U0.astype(np.float32).astype(np.float64)
        M0 = P.M0.astype(np.float32).astype(np.float64)
        _, _, f_als = oracle.als_run(Ptr.R, Ptr.Rt, M0, Ptr.lam, args.iters)
        print("n_f %d: ALS done (%.0fs)" % (n_f, time.time() - t0), flush=True)
        o = oracle.NcgOracle(Ptr.R, Ptr.Rt, n_f, Ptr.lam)
        s = o.init(U0, M0)
        f_ncg, trials = [o.f(s.x)], []
        for k in range(args.iters):
            o.step(s)
            f_ncg.append(o.f(s.x))
            trials.append(int(s.trials))
            print("n_f %d: ALS-NCG iteration %d f=%.15g (%.0fs)" % (n_f, k + 1, f_ncg[-1], time.time() - t0),
                  flush=True)
        U, M = o.split(s.x)
        pred = np.einsum("ij,ij->i", U[hr], M[hc])
        rmse = float(np.sqrt(np.mean((pred - hv.astype(np.float64)) ** 2)))
        su, sm = sample_rows(P.n_u, P.n_m)
        out["configs"][str(n_f)] = {
            "n_f": n_f, "lambda": Ptr.lam, "train_nnz": Ptr.nnz, "held_out": int(hv.size),
            "csr_digest": Ptr.R.digest(), "als_f": [float(v) for v in f_als],
            "als_ncg_f": [float(v) for v in f_ncg], "als_ncg_trials": trials,
            "als_ncg_restarts": int(s.restarts), "als_ncg_safeguards": int(s.safeguards),
            "heldout_rmse": rmse, "sample_users": su.tolist(), "sample_items": sm.tolist(),
            "U_sample": U[su].tolist(), "M_sample": M[sm].tolist()}
    with open(OUT + ".tmp", "w") as fh:
        json.dump(out, fh)
    os.replace(OUT + ".tmp", OUT)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
