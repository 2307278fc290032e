"""Writes igf_gz_quadrature.txt: the IGF z-kernel of Sec. 3 by 40-digit quadrature.

The kernel g_z(w) = (1/hz) int_{-hz}^{hz} (1 - |s|/hz) exp(-kappa |w - s|) ds
(the hat-function integral of Eq. 13-14, whose closed form is Eq. 15) depends
only on x = kappa hz and n = w / hz, so it is tabulated with hz = 1.  Values
come from oracle.igf_quad.gz_quad alone (mpmath, 40 digits); nothing here
touches the GPU library.  Run from the repository root:

    python tests/golden/make_igf_golden.py
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.igf_quad import gz_quad  # noqa: E402

X = ["1e-8", "1e-4", "0.01", "0.3", "0.49", "0.51", "1", "3.1", "12", "40"]
N = [0, 1, 2, 3, 7, 20]


def main():
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "igf_gz_quadrature.txt")
    with open(out, "w") as f:
        f.write("# IGF z-kernel g_z at w = n hz, hz = 1, kappa = x (Sec. 3, Eq. 13-15), by 40-digit\n")
        f.write("# quadrature of the hat-function integral (tests/golden/make_igf_golden.py).\n")
        f.write("# columns: x  n  g_z\n")
        for xs in X:
            for n in N:
                v = gz_quad(xs, n, 1)
                if v < 1e-290:      # below the FP64 normal range: not a useful check
                    continue
                f.write("%s %d %s\n" % (xs, n, format(float(v), ".17e")))
    print("wrote", out)


if __name__ == "__main__":
    main()
