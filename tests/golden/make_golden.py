"""Writes the regression fixtures in this folder.  Calls only the oracle.

cavity_5x6x7_lid.txt: a 5x6x7 cavity with static walls on five faces and the
+y face moving at (0.05, 0, 0), tau = 0.6, started from rest (rho = 1, u = 0),
after 6 plain steps; one line per cell (x-slowest, z-fastest): rho |u|.

Run:  python -m tests.golden.make_golden
"""
import os

import numpy as np

import oracle
from oracle import MOVING_WALL, WALL

HERE = os.path.dirname(os.path.abspath(__file__))


def cavity_case():
    o = oracle.Oracle((5, 6, 7), 0.6, faces=(WALL, WALL, WALL, MOVING_WALL, WALL, WALL), wall_u=(0.05, 0.0, 0.0))
    f = o.run(o.init(), 6)
    rho, _, unorm = o.macro(f)
    return rho, unorm


def load_fixture(path):
    return np.loadtxt(path, comments="#")


def main():
    rho, unorm = cavity_case()
    path = os.path.join(HERE, "cavity_5x6x7_lid.txt")
    with open(path, "w") as fh:
        fh.write("# oracle: 5x6x7 cavity, +y lid u=(0.05,0,0), tau=0.6, 6 steps from rest; columns rho |u|\n")
        for r, u in zip(rho.ravel(), unorm.ravel()):
            fh.write(f"{r:.17e} {u:.17e}\n")


if __name__ == "__main__":
    main()
