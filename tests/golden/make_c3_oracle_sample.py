#!/usr/bin/env python3
"""Writes c3_membrane512_oracle_sample.npz: a seeded sample of the FP64
oracle's solution of the 512^3 membrane pressure system.

The system is the benchmarked one (Sec. 2.1: the pressure Poisson equation of
the fractional step; Sec. 2.5, modules 1-3: classification, ghost rows and the
solve): a 512^3 tanh-stretched grid (largest adjacent width ratio 1.05), the
seeded cambered plate of 40,000 triangles with ghost unknowns on both sides,
and the seeded uniform-noise right-hand side.  The oracle classifies, builds
the ghost rows, assembles, solves the pinned system to a relative residual of
1e-13 and removes the volume-weighted fluid mean (the gauge).  Stored: the
gauged values at 65,536 cells and 4,096 membrane ghost unknowns drawn by a
seeded generator, the norm of the whole gauged solution over the fluid cells
and over the membrane unknowns, and the oracle's iteration count, final
residual and recursive-residual history (so the iterations the oracle needs
to reach 1e-8 are known).  Only the oracle computes; the input generators hold none of the
method's arithmetic.  Needs about 16 GB of memory and, with 8 threads, about
15 minutes.

    python tests/golden/make_c3_oracle_sample.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2605_04335_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_membrane512_oracle_sample.npz")
N_CELLS, N_MEM, SEED = 65536, 4096, 2605


def main():
    t0 = time.time()
    p = W.membrane_case(512)
    S = oracle.setup(p.xf, p.yf, p.zf, p.bodies)
    print("set-up %.0f s: %d membrane ghost unknowns" % (time.time() - t0, S.st.nm), flush=True)
    t0 = time.time()
    xg, b, x, info = oracle.solve_problem(S, p.f, tol=1e-13, maxit=400)
    print("solve %.0f s: rc %d, %d iterations, relative residual %.3e" % (time.time() - t0, info.rc, info.iters,
                                                                         info.relres), flush=True)
    assert info.rc == 0 and info.relres <= 1e-13
    N = S.N
    fluid = (S.flags & oracle.F_SOLID) == 0
    rng = np.random.default_rng(SEED)
    cells = np.sort(rng.choice(np.nonzero(fluid)[0], N_CELLS, replace=False)).astype(np.int64)
    mem = np.sort(rng.choice(S.st.nm, min(N_MEM, S.st.nm), replace=False)).astype(np.int64)
    np.savez_compressed(OUT, cells=cells, cell_values=xg[cells], mghost=mem, mghost_values=xg[N + mem],
                        norm_fluid=np.linalg.norm(xg[:N][fluid]), norm_mghost=np.linalg.norm(xg[N:]),
                        n_mghost=S.st.nm, iterations=info.iters, rel_residual=info.relres, tol=1e-13, hist=info.hist,
                        flags_sum=int(S.flags.astype(np.int64).sum()))
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
