"""Writes carpet_stokes.json: the continuum (Stokes) permeability of the
level-3 Sierpinski carpet of Sec. 4.1 (Fig. 2a), computed by the lattice
Boltzmann reference in oracle/stokes_lbm.py at two resolutions, with the
same reference's plane-channel error as a measure of its accuracy.

    python tests/golden/make_carpet_stokes.py      (about 8 minutes on 8 CPU cores)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))
from oracle.stokes_lbm import stokes_permeability  # noqa: E402
from paper_1712_01132_amd import geometry  # noqa: E402


def main():
    out = {"method": "D2Q9 BGK lattice Boltzmann, tau = 1, Guo body force, full-way bounce-back",
           "units": "k_px2 in pixel^2; k_over_L2 normalised by L^2 with L = N1 pixels (the paper's k)"}
    H = 20
    ch = np.zeros((H + 2, 8), np.uint8)
    ch[0] = ch[-1] = 1
    k, st = stokes_permeability(ch, threads=8)
    exact = H ** 2 / 12.0 * H / (H + 2)
    out["channel_H20"] = {"k_px2": k, "poiseuille_px2": exact, "rel_error": k / exact - 1, "steps": st}
    print(out["channel_H20"], flush=True)
    for n in (270, 540):
        t0 = time.time()
        c = geometry.sierpinski_carpet(3, n)
        k, st = stokes_permeability(c, threads=8, check=2000, rtol=1e-7)
        out["carpet_%d" % n] = {"k_px2": k, "k_over_L2": k / n ** 2, "porosity": float(1 - c.mean()),
                                "steps": st, "seconds": round(time.time() - t0, 1)}
        print(n, out["carpet_%d" % n], flush=True)
    with open(os.path.join(HERE, "carpet_stokes.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
