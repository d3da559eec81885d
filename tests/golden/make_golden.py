"""Write the stored oracle results used by the full-size (4088x4088) checks.

Calls only the CPU FP64 oracle and the synthetic generator:
  c3_seed1003_theta_f64.npy    theta* of the 4088^2 pair (seed 1003), FP64 inputs
  c3_seed1003_theta_f32in.npy  theta* of the same pair with both images rounded
                               to float32 first (what the FP32C mode receives)
  bench_c3_theta_f64.npy       theta* of the benchmark's 4088^2 pairs (seeds
  bench_c3_theta_f32in.npy     3000 .. 3000+B-1), one row per seed, both input
                               precisions; the benchmark compares every timed
                               pair with these and recomputes D* from them
Run:  python tests/golden/make_golden.py [--bench B]
(about a minute per 4088^2 pair on 8 cores).
"""
import argparse
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

BENCH_SEED0 = 3000


def thetas(p):
    """theta* for FP64 inputs and for float32-rounded inputs."""
    out = {}
    for tag, cast in (("f64", np.float64), ("f32in", np.float32)):
        s = p.sci.astype(cast).astype(np.float64)
        r = p.tmpl.astype(cast).astype(np.float64)
        om, be = oracle.normal_system_fft(s, r, p.mask, p.w, p.dk, p.db)
        th = oracle.solve(om, be)
        out[tag] = th
        print(tag, "n =", th.size, "rho =", np.linalg.norm(be - om @ th) / np.linalg.norm(be), flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--bench", type=int, default=0, help="also write theta* of the first B benchmark pairs")
    ap.add_argument("--skip-test-pair", action="store_true")
    args = ap.parse_args()
    if not args.skip_test_pair:
        th = thetas(synth.pair_c3(seed=1003))
        for tag, v in th.items():
            np.save(os.path.join(HERE, f"c3_seed1003_theta_{tag}.npy"), v)
    if args.bench > 0:
        rows = {"f64": [], "f32in": []}
        for i in range(args.bench):
            print("bench pair", BENCH_SEED0 + i, flush=True)
            th = thetas(synth.pair_c3(seed=BENCH_SEED0 + i))
            for tag in rows:
                rows[tag].append(th[tag])
        for tag, v in rows.items():
            np.save(os.path.join(HERE, f"bench_c3_theta_{tag}.npy"), np.stack(v))


if __name__ == "__main__":
    main()
