"""Writes analytic.json: mathematical constants used as pins, computed with mpmath only
(no code from oracle/ or the GPU package). Run: python tests/golden/make_analytic.py"""
import json
import os

import mpmath as mp

mp.mp.dps = 20


def box_F_numeric(a, b, c):
    """int_{[0,a]x[0,b]x[0,c]} dV/|y|: the z-integral done exactly (asinh(c/r)), the
    remaining 2-D integral by mpmath quadrature."""
    f = lambda x, y: mp.asinh(c / mp.sqrt(x * x + y * y))
    return mp.quad(f, [0, a], [0, b])


def main():
    out = {
        "_citation": "Box Coulomb integral: the truncated kernel's zero mode U_0 = (1/(4pi)) "
                     "int_{D_2L} dy/|y| (Sec. 2.2, eq. FUk at k = 0) = (2/pi) F(2ax, 2ay, 2az).",
        "F_1_1_1": mp.nstr(box_F_numeric(1, 1, 1), 20),
        "F_16_16_8": mp.nstr(box_F_numeric(16, 16, 8), 20),
    }
    path = os.path.join(os.path.dirname(__file__), "analytic.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
