"""Pin of the face-velocity cap (reading R6 of the revisions of Sect. 2.1.1): each
velocity component of a face limit is capped in magnitude by the larger magnitude of
that component's mean velocity in the two cells sharing the face, plus sqrt(g h_tol).

Two cells in a row on a flat bed, no limiter flags at play (flat bed: the revision
leaves depths and velocities as they are). Cell A's east face limit has a depth just
above h_tol and a finite discharge, so its velocity would be about 90 m/s; cell B is
slow. The mean-depth rate L0 of each cell is then fixed by the two mass fluxes of its
faces: at the interior face the HLL flux (the oracle's HLL, pinned on its own) of A's
capped east limit and B's west limit; at the open (transmissive) edge faces each
limit's own physical mass flux h u, the ghost being a copy (in y the north and south
limits are equal and cancel).
"""
import numpy as np
import pytest

import oracle
from oracle import Oracle
from paper_2107_02750_amd import scenarios as S

G, HT, DX = 9.80665, 1e-3, 2.0
S3 = np.sqrt(3.0)


def cap(u, ua, ub):
    m = max(abs(ua), abs(ub)) + np.sqrt(G * HT)
    return min(max(u, -m), m)


@pytest.mark.parametrize("uB", [0.1, -0.7, 2.0])
def test_face_velocity_cap_sets_the_interior_mass_flux(uB):
    hA, hA1, qA, qA1 = 0.5, -(0.5 - 0.004) / S3, 0.2, 0.1
    hB, qB = 0.3, 0.3 * uB
    vA = 0.05  # a transverse velocity in A, also capped at the face
    P = np.zeros((9, 1, 2))
    P[0, 0] = [hA, hB]
    P[1, 0, 0] = hA1
    P[3, 0] = [qA, qB]
    P[4, 0, 0] = qA1
    P[6, 0, 0] = hA * vA
    sc = S.Scenario("cap", 2, 1, DX, np.zeros((2, 3)), S.MODE_PLANES, P, h_tol=HT)
    o = Oracle(sc)
    L, _, _ = o.operator(P, 0.0)
    uA0, uB0 = qA / hA, uB
    # A's east limit: depth 0.004 m, raw velocity (qA + sqrt3 qA1) / 0.004, about 93 m/s
    hE = hA + S3 * hA1
    uE_raw = (qA + S3 * qA1) / hE
    assert uE_raw > 50.0
    uE = cap(uE_raw, uA0, uB0)
    vE = cap(hA * vA / hE, vA, 0.0)
    FE = oracle.hll(G, hE, uE, vE, hB, uB, 0.0)[0]
    # A's west limit at the open edge (cap from A alone), B's east limit at the other
    hW = hA - S3 * hA1
    uW = cap((qA - S3 * qA1) / hW, uA0, uA0)
    FW = hW * uW
    FB_east = hB * cap(uB, uB0, uB0)
    assert L[0, 0, 0] == pytest.approx(-(FE - FW) / DX, rel=1e-12, abs=1e-13)
    assert L[0, 0, 1] == pytest.approx(-(FB_east - FE) / DX, rel=1e-12, abs=1e-13)
    # without the cap the interior mass flux would differ by more than 0.4 m^2/s
    F_raw = oracle.hll(G, hE, uE_raw, hA * vA / hE, hB, uB, 0.0)[0]
    assert abs(F_raw - FE) > 0.4
