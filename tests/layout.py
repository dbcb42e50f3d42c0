"""Test-side conversion between the oracle's factor planes, [E][6][N^3]
(one plane per factor), and the library's planes of factor pairs,
[E][3][N^3][2] ((g1,g2), (g3,g4), (g5,g6) per node).  Plain reshapes: no
arithmetic of the method."""
import numpy as np


def pairs(G):
    """[E, 6, N^3] -> [E, 3, N^3, 2] (same dtype, contiguous)."""
    G = np.asarray(G)
    E, six, N3 = G.shape
    assert six == 6
    return np.ascontiguousarray(G.reshape(E, 3, 2, N3).transpose(0, 1, 3, 2))


def planes(Gp, N3):
    """The inverse of pairs for 6*E*N3 values in pair layout."""
    Gp = np.asarray(Gp).reshape(-1, 3, N3, 2)
    return np.ascontiguousarray(Gp.transpose(0, 1, 3, 2).reshape(-1, 6, N3))
