"""Writes standin_contours.json: for each sparse-shaped stand-in of Table 1
(pencilgen.sparse_standin), a circle around about 20 of its eigenvalues, the
count inside and those reference eigenvalues, chosen from the dense reference
spectrum.  With --banded, the same for the banded variants of the stand-ins
(non-zeros within a band of half-width ceil(nnz(A)/n)), written to
standin_banded_contours.json.  Calls the oracle only (oracle.dense_eigenvalues,
oracle.standin_contour).

    python tests/golden/make_standin_contours.py [--banded]
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import pencilgen as pg  # noqa: E402
from oracle import gfeast as o  # noqa: E402


def main():
    banded = "--banded" in sys.argv
    out = {}
    for k in range(1, len(pg.TABLE1) + 1):
        name, A, B, _ = pg.sparse_standin(k, banded=banded)
        lam = o.dense_eigenvalues(A, B)
        c, r, s, gap = o.standin_contour(lam)
        ins = lam[abs(lam - c) < r]
        out[str(k)] = {"name": name, "n": A.shape[0], "center": [c.real, c.imag], "radius": r,
                       "s": s, "gap": gap, "finite_eigenvalues": int(lam.size),
                       "inside": [[z.real, z.imag] for z in ins]}
        print(k, name, "s", s, "gap %.3f" % gap, flush=True)
    fname = "standin_banded_contours.json" if banded else "standin_contours.json"
    with open(os.path.join(HERE, fname), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
