"""Rounding bound between two evaluations of the CIC deposit that add the
same terms in different orders.

Both the oracle and the library form every particle's corner weight
((Wz*Wy)*Wx) with the same operations, so their vertex sums A_v hold the same
n_v non-negative terms (n_v = particles in the eight cells around vertex v)
and differ only in association: |A_v - A'_v| <= 2 gamma(n_v) * sum_v, with
gamma(n) = n u / (1 - n u), u = 2^-53 (Higham, Accuracy and Stability of
Numerical Algorithms, 2nd ed., Sec. 4.2).  Scaling by q/h^3 and adding the
background round once each; the zero-mean projection subtracts a mean that
both sides sum over all vertices in their own order.  The per-vertex part of
the difference is bounded by e_v below; the mean's part is one constant for
all vertices, bounded by e_mean."""
import numpy as np

U = 2.0 ** -53


def gamma(n):
    n = np.asarray(n, dtype=np.float64)
    return n * U / (1.0 - n * U)


def vertex_counts(N, cell_counts):
    """n_v: particles in the eight cells (v - {0,1}^3) around each vertex."""
    c = np.asarray(cell_counts, dtype=np.float64).reshape(N, N, N)
    out = np.zeros_like(c)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                out += np.roll(c, shift=(dz, dy, dx), axis=(0, 1, 2))
    return out.ravel()


def deposit_bounds(N, rho_e, rho_bg, b, cell_counts):
    """(e_v, e_mean) for the zero-mean deposit b = rho_e + rho_bg - mean."""
    n_v = vertex_counts(N, cell_counts)
    re = np.abs(np.asarray(rho_e))
    bv = np.abs(np.asarray(rho_e) + rho_bg)
    e_pre = (2.0 * gamma(n_v) + 4.0 * U) * re + 2.0 * U * bv
    n3 = N ** 3
    e_mean = e_pre.mean() + 2.0 * gamma(n3) * bv.mean()
    e_v = e_pre + 2.0 * U * np.abs(np.asarray(b))
    return e_v, e_mean


def check_deposit(N, got, ref_b, rho_e, rho_bg, cell_counts):
    """Assert that got - ref_b is within the bound: its spread over the
    vertices by the per-vertex part, its mean by the mean's part."""
    d = np.asarray(got) - np.asarray(ref_b)
    e_v, e_mean = deposit_bounds(N, rho_e, rho_bg, ref_b, cell_counts)
    c = d.mean()
    assert abs(c) <= e_mean + e_v.max(), (c, e_mean)
    # d_v = c_exact + p_v with |p_v| <= e_v: every pair differs by at most
    # e_v + e_w
    assert d.max() - d.min() <= 2.0 * e_v.max(), (d.max() - d.min(), e_v.max())
    assert np.all(np.abs(d - c) <= e_v + e_v.max()), np.max(np.abs(d - c) - e_v)
    return float(np.abs(d - c).max()), float(e_v.max())
