"""Writes radial_k160.txt: the separation-of-variables mode coefficients
b_n H_n(kR), n = 0..nmax, of the oracle (oracle/radial.py) for the radial
contrast q = 0.4 exp(-r^2 / 0.2^2) (support truncated at r = 1, tail
<= 1.4e-11 there), k = 160, R = 2.  Used by tests/test_gpu_fullsize.py for the
largest grid tested (128 x 128 leaves).
Run: python tests/golden/make_radial_k160.py"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.radial import mode_coefficients  # noqa: E402

K, AMP, SIG, A, R = 160.0, 0.4, 0.2, 1.0, 2.0

if __name__ == "__main__":
    c = mode_coefficients(K, lambda r: AMP * np.exp(-r * r / SIG ** 2), A, R)
    with open(os.path.join(HERE, "radial_k160.txt"), "w") as f:
        f.write("# b_n H_n(kR) for q = 0.4 exp(-r^2/0.04), k = 160, R = 2 (oracle/radial.py)\n")
        f.write("# columns: n, real, imag\n")
        for n, v in enumerate(c):
            f.write(f"{n} {v.real:.17e} {v.imag:.17e}\n")
