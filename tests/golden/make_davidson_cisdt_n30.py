"""Write davidson_cisdt_n30.txt: the two lowest energies of the CISDT
workload with 30 orbitals (recipe A, seed 1, 30 bohr box, 60 auxiliary
points, tau = 1e-14) from the CPU oracle's textbook Davidson (residual
<= 1e-9 per root).  Calls only oracle/ and isci_inputs/; run from the
repository root:  python tests/golden/make_davidson_cisdt_n30.py"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from isci_inputs import workload  # noqa: E402

NROOTS = 2
TOL = 1e-9


def main():
    W = workload("cisdt_n30")
    h, eri = W.integrals()
    S = O.Space(W.norb, W.nalpha, W.nbeta, W.level)
    t0 = time.time()
    e, _, rn = O.davidson(S, h, eri, W.tau, nroots=NROOTS, tol=TOL, maxiter=600)
    assert np.all(rn <= TOL), rn
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "davidson_cisdt_n30.txt")
    with open(out, "w") as f:
        f.write("# Lowest energies (Eh, electronic) of the CISDT workload, 30 orbitals, recipe A seed 1,\n")
        f.write(f"# box 30, 60 auxiliary points, tau {W.tau:g}, dim {S.dim}: the CPU oracle's textbook\n")
        f.write(f"# Davidson on its Slater-Condon sigma, residual norms {', '.join(f'{x:.1e}' for x in rn)}\n")
        f.write(f"# (written by tests/golden/make_davidson_cisdt_n30.py in {time.time() - t0:.0f} s)\n")
        for x in e:
            f.write(f"{x:.17g}\n")
    print(open(out).read())


if __name__ == "__main__":
    main()
