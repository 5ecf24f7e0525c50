"""Writes coupling_high_degree.txt: sampled coupling coefficients A^p_q(l, m) at high degrees,
computed by the oracle alone (oracle.slsht.oracle_coupling_exact: the sum over l' of f
times the exact Gaunt integral, the triple product T of Eq:harmonic_formulation) from seeded
inputs (paper_1207_5558_amd.inputs).

Exact integrals rather than the oracle's quadrature, whose rounding reaches 1e-12 relative
at l = 300-400; either takes too long for a test.  The GPU test
(tests/test_gpu_parity.py::test_coupling_high_degree_golden) regenerates the same inputs
and compares the library's coupling with these entries.

    python tests/golden/make_coupling_high_degree.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.slsht import oracle_coupling_exact  # noqa: E402
from paper_1207_5558_amd.inputs import draw_coefficients  # noqa: E402

# (L_f, L_h, degree l, seed, sampled orders m, sampled (p, q) or None for all)
CASES = [
    (400, 6, 399, 401, (-399, -398, -250, -37, -1, 0, 1, 2, 150, 397, 398, 399), None),
    (300, 32, 300, 302, (-300, -151, -2, 0, 3, 120, 299, 300),
     ((0, 0), (1, -1), (5, 3), (12, -12), (17, 0), (20, 19), (31, -31), (31, 0), (31, 30),
      (26, -7))),
]


def main():
    lines = ["# sampled A^p_q(l, m) from oracle_coupling_exact; f = draw_coefficients(",
             "#   np.random.default_rng(seed), L_f, 2.0, True); written by make_coupling_high_degree.py",
             "# L_f L_h seed l m p q Re Im"]
    for L_f, L_h, l, seed, ms, pqs in CASES:
        f = draw_coefficients(np.random.default_rng(seed), L_f, 2.0, True)
        if pqs is None:
            pqs = [(p, q) for p in range(L_h) for q in range(-p, p + 1)]
        for m in ms:
            for p, q in pqs:
                v = oracle_coupling_exact(f, L_f, l, m, p, q)
                lines.append(f"{L_f} {L_h} {seed} {l} {m} {p} {q} {v.real:.17e} {v.imag:.17e}")
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "coupling_high_degree.txt")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(f"wrote {len(lines) - 3} entries to {out}")


if __name__ == "__main__":
    main()
