#!/usr/bin/env python3
"""Degree sweep of the eigensolver loop: for each filter degree m, the cycles
of bounds, filter and Rayleigh-Ritz (abi_chebfi_solve) from the same seeded
start block until the lowest `nconv` residual norms are <= tol; prints one
JSON line per degree with the cycles, wall time and H applications used.

This is the trade-off the paper studies between the filter degree, the
number of outer iterations and the time to solution (section "Chebyshev
filtering: influence of the polynomial degree").  With --lobpcg b:k ... the
same start block is also solved by block LOBPCG with b blocks and k line
minimisations per pass (abi_lobpcg_solve), the paper's comparison solver;
--paw adds the PAW-like overlap S to the system.

    python -m paper_2604_11139_amd.sweep --config 2 --degrees 4 6 8 10 12 16
    python -m paper_2604_11139_amd.sweep --config 2 --degrees 10 --lobpcg 4:4 1:4 --paw
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, default=2, choices=[1, 2, 3])
    ap.add_argument("--degrees", type=int, nargs="+", default=[4, 6, 8, 10, 12, 16])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--nconv-frac", type=float, default=0.8)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-cycles", type=int, default=60)
    ap.add_argument("--refine-degree", type=int, default=4)
    ap.add_argument("--lobpcg", nargs="*", default=[],
                    help="block LOBPCG runs as nblocks:nline (FP64 blocks)")
    ap.add_argument("--max-passes", type=int, default=60)
    ap.add_argument("--paw", action="store_true", help="add the PAW-like overlap S")
    args = ap.parse_args()

    import torch

    import workloads as W
    from paper_2604_11139_amd import binding as B

    s = W.make_system(args.config, q_scale=W.PAW_Q_SCALE if args.paw else 0.0)
    mixed = args.precision == "mixed"
    with B.System(s, precision=B.ABI_PREC_MIXED if mixed else B.ABI_PREC_FP64) as g:
        X0 = torch.from_numpy(W.random_block(g.npw, s.nband, s.tag).T).to("cuda")
        v0 = torch.from_numpy(W.random_vector(g.npw, s.tag)).to("cuda")
        if mixed:
            X0 = X0.to(torch.complex64)
        nconv = max(1, int(args.nconv_frac * s.nband))
        for m in args.degrees:
            X = X0.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ev, res, info = g.solve(X, v0, m, args.max_cycles, nconv, args.tol,
                                    args.refine_degree if mixed else 0)
            wall = time.perf_counter() - t0
            happ = s.nband * (m * info["cycles"] + args.refine_degree * info["refine_cycles"])
            print(json.dumps({
                "config": args.config, "precision": args.precision, "degree": m,
                "nconv": nconv, "tol": args.tol, **info, "wall_s": round(wall, 3),
                "h_applications_in_filters": happ,
                "max_residual_nconv": float(res[:nconv].max()),
                "lowest_eval": float(ev[0]), "eval_nconv": float(ev[nconv - 1]),
                "paw": args.paw,
            }), flush=True)
        X64 = X0.to(torch.complex128)
        for spec in args.lobpcg:
            nb, nl = (int(v) for v in spec.split(":"))
            X = X64.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ev, res, info = g.lobpcg(X, nb, nl, args.max_passes, nconv, args.tol)
            wall = time.perf_counter() - t0
            print(json.dumps({
                "config": args.config, "solver": "lobpcg", "nblocks": nb, "nline": nl,
                "nconv": nconv, "tol": args.tol, **info, "wall_s": round(wall, 3),
                "max_residual_nconv": float(res[:nconv].max()),
                "lowest_eval": float(ev[0]), "eval_nconv": float(ev[nconv - 1]),
                "paw": args.paw,
            }), flush=True)


if __name__ == "__main__":
    main()
