"""Writes the golden fixtures of this folder from oracle/exact.py only.

bspline1d_K8_p2.txt: exact 1D mass (scaled by 1920) and stiffness matrices of
the open uniform quadratic B-spline basis with 8 elements on [0,1] (Sec. 2.3,
eqs. knot_vector, cox1/cox2; integrals of products of the 10 basis functions).
Run:  python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import exact  # noqa: E402


def main():
    M, A = exact.matrices_1d(exact.open_uniform_knots(8, 2), 2)
    lines = ["# exact 1D matrices, open uniform knots, K=8, p=2 (10 functions)",
             "# format  name:row:entries   (1920M = 1920 * int N_i N_j, A = int N_i' N_j')"]
    for i in range(10):
        lines.append("1920M:%d:%s" % (i, " ".join(str(1920 * v) for v in M[i])))
    for i in range(10):
        lines.append("A:%d:%s" % (i, " ".join(str(v) for v in A[i])))
    with open(os.path.join(HERE, "bspline1d_K8_p2.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
