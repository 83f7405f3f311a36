"""The paper's operation-count model (oracle; test infrastructure).

Sec. 5.2, eqn flopRealMF, flopComplexMF, flopRealCM, flopComplexCM: floating
point operations of one matrix-free / cell-matrix action on n_v vectors over
E cells, with the even-odd decomposition in the matrix-free counts.  The batch
factors b^(2) n_b^(2) n_b^(1) of the paper multiply to c n_v (eq batchedlayout),
so the counts below are written per real lane and multiplied by c n_v.

Pins (tests/test_oracle_flops.py): the leading-order statements of the paper
(about 12 n_p^4 per vector per cell for n_q ~ n_p; 2 n_p^6 and 6 n_p^6 for the
cell-matrix action) and the quoted quadrature ratios at FEOrder 8 (lowering
n_q = n_p + 2 to n_p saves about 1.8x; raising to n_p + 3 costs about 1.4x).
"""


def _split(n):
    return n // 2, (n + 1) // 2


def flop_mf_real(np_, nq, E, nvec, ns=0, nb1=1):
    npo, _ = _split(np_)
    nqo, _ = _split(nq)
    per = (2 * (npo * (nq + 2) + nqo * (np_ + 2)) * (np_ ** 2 + np_ * nq + nq ** 2)
           + 6 * nqo * nq ** 2 * (2 * nq + 5) + 34 * nq ** 3)
    return per * nvec * E + 2 * nq ** 3 * nb1 * E + nvec * (4 * np_ ** 3 + 1) * ns


def flop_mf_complex(np_, nq, E, nvec, ns=0, nb1=1):
    """nvec counts complex vectors; the paper's lanes are c n_v = 2 nvec."""
    npo, _ = _split(np_)
    nqo, _ = _split(nq)
    lanes = 2 * nvec
    per = (2 * (npo * (nq + 2) + nqo * (np_ + 2)) * (np_ ** 2 + np_ * nq + nq ** 2)
           + 6 * nqo * nq ** 2 * (2 * nq + 5) + 40 * nq ** 3)
    return per * lanes * E + 2 * nq ** 3 * nb1 * E + lanes * (8 * np_ ** 3 + 3) * ns


def flop_cm_real(np_, E, nvec, ns=0):
    return 2 * nvec * np_ ** 6 * E + nvec * (4 * np_ ** 3 + 1) * ns


def flop_cm_complex(np_, E, nvec, ns=0):
    return 6 * nvec * np_ ** 6 * E + 3 * nvec * (4 * np_ ** 3 + 1) * ns
