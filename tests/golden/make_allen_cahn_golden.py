"""Write the oracle's eigen-data for the 2-D Allen-Cahn Hessian (d = n^2).

Calls only the oracle (cyclic Jacobi, FP64) and the seeded input generator.
For each seed it stores, in ``allen_cahn_n{n}_seed{seed}.npz`` beside this
script: the field u, all eigenvalues ascending, and the eigenvectors of the
``nvec`` smallest eigenvalues (enough for R_k = I - 2 Q_k Q_k^T with
k < nvec), plus the Jacobi sweep count.

    python tests/golden/make_allen_cahn_golden.py --n 64 --seeds 0
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2605_24840_amd import inputs  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--eps", type=float, default=0.05)
    ap.add_argument("--seeds", type=int, nargs="+", default=[0])
    ap.add_argument("--nvec", type=int, default=8)
    args = ap.parse_args()
    for seed in args.seeds:
        t0 = time.time()
        H, u = inputs.allen_cahn_2d(args.n, args.eps, seed)
        w, V, sweeps = oracle.jacobi_eigh(H)
        out = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                           f"allen_cahn_n{args.n}_seed{seed}.npz")
        np.savez(out, u=u, w=w, V=np.ascontiguousarray(V[:, :args.nvec]), sweeps=sweeps,
                 eps=args.eps, n=args.n, seed=seed)
        print(f"seed {seed}: d={H.shape[0]} sweeps={sweeps} lam[:6]={w[:6]} "
              f"({time.time() - t0:.0f}s, {oracle.oracle_threads()} threads) -> {out}", flush=True)


if __name__ == "__main__":
    main()
