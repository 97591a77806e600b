"""Hand-worked betweenness values (tests/golden/hand_worked_bc.txt)."""
import os

import numpy as np
import pytest

import graphgen as gg
import oracle

O = oracle.load()
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hand_worked_bc.txt")


def cases():
    out = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, n, edges, vals = [x.strip() for x in line.split(";")]
        e = [tuple(map(int, ab.split("-"))) for ab in edges.split(",")]
        out.append((name, int(n), e, [float(x) for x in vals.split()]))
    return out


@pytest.mark.parametrize("name,n,edges,want", cases(), ids=[c[0] for c in cases()])
def test_hand_worked(name, n, edges, want):
    e = np.array(edges)
    g = gg.from_edges(n, e[:, 0], e[:, 1])
    assert np.allclose(O.bc_exact(g), want, rtol=1e-15, atol=0)
