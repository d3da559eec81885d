"""Write the stored oracle results used by the full-size (4088x4088) GPU parity test.

Calls only the CPU FP64 oracle and the synthetic generator:
  c3_seed1003_theta_f64.npy   theta* of the 4088^2 pair (seed 1003), FP64 inputs
  c3_seed1003_theta_f32in.npy theta* of the same pair with both images rounded
                              to float32 first (what the FP32C mode receives)
Run:  python tests/golden/make_golden.py   (about a minute on 8 cores)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def main():
    p = synth.pair_c3(seed=1003)
    for tag, cast in (("f64", np.float64), ("f32in", np.float32)):
        s = p.sci.astype(cast).astype(np.float64)
        r = p.tmpl.astype(cast).astype(np.float64)
        om, be = oracle.normal_system_fft(s, r, p.mask, p.w, p.dk, p.db)
        th = oracle.solve(om, be)
        np.save(os.path.join(HERE, f"c3_seed1003_theta_{tag}.npy"), th)
        print(tag, "n =", th.size, "rho =", np.linalg.norm(be - om @ th) / np.linalg.norm(be))


if __name__ == "__main__":
    main()
