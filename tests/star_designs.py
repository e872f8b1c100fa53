"""Designed increments for Algorithm 2 (TT-ICE*, Sec. 3.3) whose decisions
have closed-form outcomes.  Input construction only: no TT-ICE arithmetic.

Every design is a stream of order-2 tensors (n_1 x n_2, d = 2) built from
seeded orthonormal bases e_1.. of R^{n_1} and f_1.. of R^{n_2}.  Its first
increment is one tensor e_1 f_1^T, which gives the cores U_1 = [e_1],
U_2 = [f_1] (ranks [1, 1, 1, 1]); the approximation of any tensor Y with
those cores is (e_1^T Y f_1) e_1 f_1^T, so the error of a tensor built from
other basis products is exactly the norm of those products.
"""
import numpy as np


def bases(n1, n2, seed):
    rng = np.random.default_rng(seed)
    e, _ = np.linalg.qr(rng.standard_normal((n1, n1)))
    f, _ = np.linalg.qr(rng.standard_normal((n2, n2)))
    return e, f


def outer(e, f, i, j):
    return np.multiply.outer(e[:, i], f[:, j])


def dc_share_design(seed=0):
    """eps = 0.1.  Second increment:
      frame 0 (in D_C): a e_1 f_1^T + b e_3 f_3^T, a^2 = 99.19, b^2 = 0.81
                        (norm^2 100, relative error 0.09 <= eps);
      frame 1 (in D):   s_1 e_2 f_2^T + s_2 e_4 f_4^T, s_1^2 = 0.3, s_2^2 = 0.09
                        (relative error 1; singular values s_1 > s_2).
    Returns (dims, eps, first_increment, second_increment)."""
    n1, n2 = 6, 5
    e, f = bases(n1, n2, seed)
    first = outer(e, f, 0, 0)[None]
    y0 = np.sqrt(99.19) * outer(e, f, 0, 0) + np.sqrt(0.81) * outer(e, f, 2, 2)
    y1 = np.sqrt(0.3) * outer(e, f, 1, 1) + np.sqrt(0.09) * outer(e, f, 3, 3)
    return (n1, n2), 0.1, first, np.stack([y0, y1])


def batch_rule_design(seed=1):
    """eps = 0.1.  Second increment:
      frame 0: a e_1 f_1^T + b e_3 f_3^T, a^2 = 99.75, b^2 = 0.25
               (norm^2 100, relative error 0.05);
      frame 1: s e_2 f_2^T, s^2 = 0.01 (relative error 1).
    The mean of the relative errors is 0.525 > eps; the batch relative error
    (eq:batchrelativeerror) is sqrt(0.26 / 100.01) = 0.0510 <= eps."""
    n1, n2 = 6, 5
    e, f = bases(n1, n2, seed)
    first = outer(e, f, 0, 0)[None]
    y0 = np.sqrt(99.75) * outer(e, f, 0, 0) + np.sqrt(0.25) * outer(e, f, 2, 2)
    y1 = np.sqrt(0.01) * outer(e, f, 1, 1)
    return (n1, n2), 0.1, first, np.stack([y0, y1])


def occupancy_design(seed=2):
    """n_1 = 5, n_2 = 3, eps = 0.1.  First increment: four tensors
    c_b e_b g^T (b = 1..4, c = 4, 3, 2, 1, g a unit vector of R^3), which make
    core 1 of rank 4 out of 5 rows: occupancy exactly 4/5 = 0.8 (the double
    nearest 0.8 on both sides of the comparison).  Second increment: one
    tensor e_5 g'^T entirely outside the span of core 1."""
    n1, n2 = 5, 3
    e, f = bases(n1, n2, seed)
    first = np.stack([c * outer(e, f, b, 0) for b, c in enumerate((4.0, 3.0, 2.0, 1.0))])
    second = outer(e, f, 4, 1)[None]
    return (n1, n2), 0.1, first, second
