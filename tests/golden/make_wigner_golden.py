"""Write wigner_d_mpmath.txt: reference d^l_{mk}(theta) values at moderate l.

Values come from Wigner's explicit finite sum for the small d-matrix, evaluated
with mpmath at 120 significant digits (enough to absorb the cancellation of the
alternating sum up to l = 100), i.e. the textbook definition, not a recursion.
Rerun with:  python tests/golden/make_wigner_golden.py
"""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

import mpmath  # noqa: E402

from oracle.brute import wigner_d_explicit  # noqa: E402

CASES = []
for l in (25, 50, 100):
    for m in (0, 1, 7, l // 2, l - 1, l, -3, -l):
        for k in (0, 2, 5, 16, -5):
            if abs(k) <= l and abs(m) <= l:
                for theta in ("0.01", "0.7", "1.5707963267948966", "2.9"):
                    CASES.append((l, m, k, theta))

if __name__ == "__main__":
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "wigner_d_mpmath.txt")
    with open(out, "w") as f:
        f.write("# l m k theta d^l_mk(theta) at theta rounded to binary64  (Wigner explicit sum, mpmath 120 digits)\n")
        for l, m, k, th in CASES:
            v = wigner_d_explicit(l, m, k, float(th), dps=120)  # the exact binary64 angle
            f.write("%d %d %d %s %s\n" % (l, m, k, th, mpmath.nstr(v, 25, min_fixed=1, max_fixed=0)))
    print("wrote", out, len(CASES))
