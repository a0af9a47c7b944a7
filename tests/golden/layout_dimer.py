"""Expected feature vector of an isolated dimer in the paper's feature
enumeration (GMP-Featurizer, arXiv 2303.12980, section "Examples": the probe
set is the Cartesian product of orders and sigmas, order-major, and order -1,
the local density, gives one feature without a sigma).

The dimer's features have closed forms (two atoms of one element at distance
r, centre 0): order -1 is the density sum_k B_k (1 + exp(-beta_k r^2)); order
0 is c_0(0) + c_0(r^2) (self term plus the neighbour); order l >= 1 sees the
neighbour only, F = sqrt((2l-1)!! l!) |c_l(r^2)| r^l.  Each (order, sigma)
of the golden enumeration thus has its own value, so comparing a library's
output vector with this one, position by position, pins its layout.  The
radial factors come from the oracle (test infrastructure)."""
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

DIMER_R = 1.7
B = np.array([1.3, 0.4])
BETA = np.array([0.8, 3.1])


def golden():
    with open(os.path.join(HERE, "feature_enumeration.json")) as f:
        return json.load(f)


def dimer_structure():
    pos = np.array([[0.0, 0.0, 0.0], [DIMER_R, 0.0, 0.0]])
    return pos, np.zeros(2, np.int32), np.zeros((3, 3)), 0


def expected_vector():
    """Closed-form features of atom 0 in the golden enumeration order."""
    import oracle
    fx = golden()
    q = DIMER_R ** 2
    out = []
    for l, sg in fx["features"]:
        if l == -1:
            out.append(float(np.sum(B * (1.0 + np.exp(-BETA * q)))))
        elif l == 0:
            out.append(float(oracle.radial(0, sg, B, BETA, 0.0)[0] + oracle.radial(0, sg, B, BETA, q)[0]))
        else:
            dfact = float(np.prod(np.arange(2 * l - 1, 0, -2)))
            fact = float(np.prod(np.arange(1, l + 1)))
            out.append(float(np.sqrt(dfact * fact) * abs(oracle.radial(l, sg, B, BETA, q)[0]) * DIMER_R ** l))
    return np.array(out)
