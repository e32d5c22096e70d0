"""Evaluate saved lattices against Table 1 of the paper.

Usage: python tests/golden/evaluate_table1.py DIR

DIR holds the final states written by
`python -m paper_1906_06327_amd.continuation --save-states DIR ...`
(files lattice{2,3}d_g<g>_omega<Omega>_n<n>.npy).  Each is evaluated by the
oracle's fourth-order functional (mu and E of Eqs. (e2d) / (e3d)) and
printed beside the values Table 1 prints (table1.json in this folder).
Test infrastructure: it uses the oracle.
"""
import glob
import json
import os
import re
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_1906_06327_amd import continuation as C  # noqa: E402


def main(d):
    cols = json.load(open(os.path.join(HERE, "table1.json")))["columns"]
    pat = re.compile(r"lattice(\d)d_g([0-9.e+-]+)_omega([0-9.]+)_n(\d+)\.npy$")
    for path in sorted(glob.glob(os.path.join(d, "lattice*d_*.npy"))):
        m = pat.search(os.path.basename(path))
        if not m:
            continue
        dim, g, om, n = int(m.group(1)), float(m.group(2)), float(m.group(3)), int(m.group(4))
        # the exact g of the chain entry the file name abbreviates
        g = min((c[0] for c in (C.CHAIN if dim == 2 else C.CHAIN_3D)), key=lambda v: abs(v - g))
        psi = np.load(path).astype(np.complex128)
        f = O.functional_fourth_order(O.make_params(**C.params(g, om, n, dim)), psi)
        col = next(c for c in cols if c["omega"] == om and abs(c["g2d"] - (g if dim == 2 else
                   g / (2 * np.pi / C.LAM_3D) ** 0.5)) < 1e-3 * c["g2d"])
        key = "_2d" if dim == 2 else "_3d"
        print(f"{dim}D g={g:g} Omega={om:g} n={n}: mu {f['mu']:.4f} (Table 1: {col['mu' + key]}), "
              f"E {f['energy']:.4f} (Table 1: {col['E' + key]})")


if __name__ == "__main__":
    main(sys.argv[1])
