"""Writes c3_burgers_k<K>.txt: sampled values of the oracle's waveform-relaxation iterate
for the full-size Burgers workload (n = 4096, nu = 5e-3, T = 0.5, one window, 512
uniform samples, Jacobian-corrected iteration of Secs. 2.3-2.4, rank <= 24, l = 80)
after K iterations (K = 2 and the workload's full K = 12 are stored), with the
Chebyshev-polynomial p(t), or with `spline` the piecewise-cubic p(t) of the paper's
implementation (file c3_burgers_spline_k<K>.txt).  Calls only the oracle and the seeded
input generator; the dense oracle route takes about half a minute per iteration at this
size.

    python tests/golden/make_c3_golden.py [K] [spline]
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

N_SAMPLED = 96


def sample_points(n, s, count, seed=5):
    rng = np.random.default_rng(seed)
    return rng.integers(0, n, count), rng.integers(0, s, count)


def main(K, spline=False):
    bp = synth.config_c3(K=K)
    bp.source_fit = 1 if spline else 0
    ref, hist = oracle.wr_burgers(bp, "dense", return_history=True)  # (n, s)
    ii, kk = sample_points(bp.n, bp.s, N_SAMPLED)
    tag = "spline_" if spline else ""
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"c3_burgers_{tag}k{K}.txt")
    with open(out, "w") as f:
        f.write("# Oracle waveform relaxation (Secs. 2.3-2.4, eqs. 2.10-2.20), Burgers n=4096, nu=5e-3,\n")
        f.write(f"# T=0.5, P=1, s=512 uniform samples, Jacobian-corrected, rank<=24, l=80, K={K} iterations,\n")
        f.write(f"# p(t) {'piecewise-cubic spline' if spline else 'Chebyshev least squares'}.\n")
        f.write("# Written by tests/golden/make_c3_golden.py (oracle only).\n")
        f.write("increments " + " ".join(f"{h['increment']:.17e}" for h in hist) + "\n")
        f.write("column_norms " + " ".join(f"{v:.17e}" for v in np.linalg.norm(ref, axis=0)) + "\n")
        for i, k in zip(ii, kk):
            f.write(f"value {int(i)} {int(k)} {ref[i, k]:.17e}\n")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 2, len(sys.argv) > 2 and sys.argv[2] == "spline")
