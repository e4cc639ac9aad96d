"""Writes mlp256_labels.npz: the oracle's corner labels (Sec. 3: phi' at
every grid corner, inside iff the logit is > 0) of the seeded MLP field
(seed 3: 32 spheres, 6 Fourier bands, 4 x 256 ReLU) on the 256^3 grid over
[-0.5, 0.5]^3, and the corners whose binary64 logit lies within 1e-5 of 0
(near-ties: either label is a correct binary32 evaluation).

Calls only oracle/ (the binary64 network of odc_oracle.c); about 17M network
evaluations, a few minutes on 8 host threads.  Run from the repository root:
    python tests/golden/make_mlp256_labels.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import odc_inputs as I  # noqa: E402
from oracle import oracle as O  # noqa: E402

RES, SEED, TIE = 256, 3, 1e-5


def main():
    O.build()
    t = time.time()
    m = O.Oracle(I.mlp_field(SEED), I.unit_grid(RES, 15), mlp_tie_eps=TIE,
                 topology_only=True).mesh()
    bits = np.packbits(m["corner_label"], bitorder="little")
    ties = np.nonzero(m["corner_tie"])[0].astype(np.int64)
    out = os.path.join(HERE, "mlp256_labels.npz")
    np.savez_compressed(out, res=RES, seed=SEED, tie_eps=TIE, label_bits=bits, tie_corners=ties,
                        n_edges=m["edge_id"].size, n_pairs=m["pair_face"].size,
                        n_cells=m["cell_id"].size)
    print(f"{out}: {m['corner_label'].size} corners, {int(m['corner_label'].sum())} inside, "
          f"{ties.size} near-ties, {m['edge_id'].size} crossing edges, "
          f"{m['cell_id'].size} active cells; {time.time() - t:.0f} s")


if __name__ == "__main__":
    main()
