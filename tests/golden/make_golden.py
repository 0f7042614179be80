"""Write the exact-rational golden fixtures of tests/golden/.

Calls only oracle/ (the closed-form chart of the 1D integrals and the
constant-Jacobian Kronecker form).  Run from the repository root:

    python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import closed_forms  # noqa: E402

HEADER = """# Exact H1 Gram matrix of the cube (0,2)^3 (affine map J = 2 I), order p = 3.
# Source: the 1D integral chart (2.103)-(2.114) of Section 2.8.2 combined with the
# constant-Jacobian simplification of Section 2.8.1 applied to the H1 inner product
# (2.31): det J = 8, D = I/4, so G = 8 M(x)M(x)M + 2 (K(x)M(x)M + M(x)K(x)M + M(x)M(x)K)
# with M = F^00 and K = F^11 restricted to indices 0..3, direction 1 fastest.
# Storage: LAPACK 'U' packed column-major, entry (I, J), I <= J, at I + J(J+1)/2.
# One line per stored entry: "I J numerator/denominator".
# Written by tests/golden/make_golden.py from oracle/closed_forms.py.
"""


def main():
    G = closed_forms.kron_gram("H1", 3, [[2, 0, 0], [0, 2, 0], [0, 0, 2]])
    n = G.shape[0]
    lines = [HEADER.rstrip("\n")]
    for J in range(n):
        for I in range(J + 1):
            v = G[I, J]
            lines.append(f"{I} {J} {v.numerator}/{v.denominator}")
    with open(os.path.join(HERE, "h1_cube2_p3_exact.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
