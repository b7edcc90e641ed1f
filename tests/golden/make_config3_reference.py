#!/usr/bin/env python3
"""Writes config3_cycles.json: the FP64 oracle's subspace iteration on the large
synthetic workload (cubic a = 30 bohr, E_cut = 20 Ha, 115313 plane waves, 64^3
grid, 216 atoms, 2048 bands, degree 12), four cycles of spectral bounds,
Chebyshev filter and Rayleigh-Ritz from the seeded start block, as in the
paper's filtering loop (Algorithm "Parallel Chebyshev filtering of degree k").

Stored: the bounds and Ritz values of every cycle, the residual norms of the
last cycle, and the Hellmann-Feynman density rho_p of the lowest p Ritz vectors
of the last cycle (p = the largest Ritz-value gap between bands 1000 and 1048,
so that no degenerate cluster is split) at 256 seeded grid points, with its
total (= p) and maximum.  Calls only the oracle and the input generators; run
once on a CPU (about half an hour on 8 cores, ~35 GB of memory).
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402


def main():
    t0 = time.time()
    s = W.make_system(3)
    H = O.Hamiltonian.from_system(s)
    X = W.random_block(H.npw, s.nband, s.tag)
    v0 = W.random_vector(H.npw, s.tag)
    cycles = []
    rr = None
    for cyc in range(s.cycles):
        a, b, a0 = O.filter_bounds(H, X, v0)
        Y = O.cheb_filter(H, X, s.degree, a, b, a0)
        del X
        rr = O.rayleigh_ritz(H, Y)
        del Y
        res = O.residual_norms(rr["Psi"], rr["HPsi"], rr["eval"])
        cycles.append(dict(bounds=[a, b, a0], eval=rr["eval"].tolist(),
                           max_residual=float(res.max())))
        print(f"cycle {cyc + 1}: bounds {a:.6f} {b:.6f} {a0:.6f}, "
              f"max residual {res.max():.3e}, {time.time() - t0:.0f} s", flush=True)
        X = rr["Psi"]
        last_res = res
        rr.pop("HPsi")
    ev = rr["eval"]
    lo, hi = 1000, 1048
    # ev[lo - 1 + j] is band lo + j (1-based); diff j is the gap above it
    p = lo + int(np.argmax(np.diff(ev[lo - 1:hi])))
    rho = O.density(H, rr["Psi"][:, :p])
    rng = np.random.default_rng([2604, 11139, 5])
    pts = np.sort(rng.choice(rho.size, size=256, replace=False))
    out = dict(
        workload="cubic a=30 bohr, Ecut=20 Ha, 115313 plane waves, 64^3 grid, 216 atoms, "
                 "2048 bands, degree 12, 4 cycles from the seeded start block (FP64 oracle)",
        npw=int(H.npw), nband=int(s.nband), degree=int(s.degree), cycles=cycles,
        last_residuals=last_res.tolist(), p=int(p), gap_at_p=float(ev[p] - ev[p - 1]),
        rho_points=pts.tolist(), rho_values=rho[pts].tolist(), rho_sum=float(rho.sum()),
        rho_max=float(rho.max()), max_residual_below_p=float(last_res[:p].max()),
    )
    with open(os.path.join(HERE, "config3_cycles.json"), "w") as f:
        json.dump(out, f)
    print(f"done in {time.time() - t0:.0f} s, p = {p}", flush=True)


if __name__ == "__main__":
    main()
