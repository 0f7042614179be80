"""Master-element shape functions of the hexahedral exact sequence.

Section 2.2 builds every space as tensor products of the 1D pair
(W_I^p = P^p with basis chi_i, Y_I^p = P^{p-1} with basis nu_i):

* H1      W^p:  chi_{i1} chi_{i2} chi_{i3},                 i_d in [0, p]      (2.33)
* L2      Y^p:  nu_{i1} nu_{i2} nu_{i3},                    i_d in [0, p-1]    (2.17)
* H(div)  V^p:  component a holds mu_{a,1} mu_{a,2} mu_{a,3} e_a with
                mu_{a,d} = chi if d == a else nu                                (2.51)-(2.52)
* H(curl) Q^p:  component a holds rho_{a,1} rho_{a,2} rho_{a,3} e_a with
                rho_{a,d} = nu if d == a else chi                               (2.69)-(2.70)

Flat index (0-based components a = 0, 1, 2 concatenated in that order,
i1 fastest): I = off_a + i1 + R1(a) i2 + R1(a) R2(a) i3 where R_d(a) is the
1D range of direction d in component a.  This is the ordering of the
correspondence formulas after (2.17), in (2.33)'s text, (2.53) and (2.71).

Reading taken: the paper prints dim W^p as (p1+1)(p2+2)(p3+1) in
Section 2.4; it is read as (p1+1)(p2+1)(p3+1), consistent with the index
formula of Algorithm 5.  The paper fixes no orientation or sign changes; none
are applied (broken, element-local test spaces, Section 3).

Every function returned here carries its full master-coordinate gradient,
computed by differentiating each 1D factor; grad, curl and div are then
formed from their definitions (2.30), (2.67), (2.48) by the Gram module.
"""
import numpy as np

from . import poly1d


def orders(p):
    """(p1, p2, p3) of an order given as one int (the same in every direction)
    or per direction (the non-uniform orders of the text after Algorithm 2):
    the 1D pair of direction d is (W_I^{p_d}, Y_I^{p_d}), so each formula below
    takes p_d in direction d."""
    if np.ndim(p) == 0:
        return (int(p),) * 3
    q = tuple(int(x) for x in p)
    if len(q) != 3:
        raise ValueError(f"need three orders, got {p}")
    return q


def ranges(space, p):
    """R[a][d]: number of 1D functions of direction d in component a."""
    q = orders(p)
    if space == "H1":
        return [[q[d] + 1 for d in range(3)]]
    if space == "L2":
        return [[q[d] for d in range(3)]]
    if space == "HDIV":
        return [[q[d] + 1 if d == a else q[d] for d in range(3)] for a in range(3)]
    if space == "HCURL":
        return [[q[d] if d == a else q[d] + 1 for d in range(3)] for a in range(3)]
    raise ValueError(space)


def factor_kinds(space):
    """K[a][d] in {'chi', 'nu'}: which 1D family builds direction d of component a."""
    if space == "H1":
        return [["chi"] * 3]
    if space == "L2":
        return [["nu"] * 3]
    if space == "HDIV":
        return [["chi" if d == a else "nu" for d in range(3)] for a in range(3)]
    if space == "HCURL":
        return [["nu" if d == a else "chi" for d in range(3)] for a in range(3)]
    raise ValueError(space)


def dimension(space, p):
    return sum(int(np.prod(r)) for r in ranges(space, p))


def basis_index(space, p):
    """Array idx[n, 4] = (a, i1, i2, i3) in flat order."""
    rows = []
    for a, R in enumerate(ranges(space, p)):
        for i3 in range(R[2]):
            for i2 in range(R[1]):
                for i1 in range(R[0]):
                    rows.append((a, i1, i2, i3))
    return np.array(rows, dtype=np.int64)


def flat_index(space, p, a, i1, i2, i3):
    R = ranges(space, p)
    off = sum(int(np.prod(R[c])) for c in range(a))
    return off + i1 + R[a][0] * i2 + R[a][0] * R[a][1] * i3


def evaluate(space, p, xi, subset=None):
    """Evaluate basis functions at points xi[Q, 3].

    Returns (comp[n], val[Q, n], grad[Q, n, 3]) where function I is
    val[:, I] * e_{comp[I]} (scalar spaces: comp = 0) and grad[:, I, e] is the
    derivative of val[:, I] with respect to xi_e.  `subset` restricts the
    output to the given flat indices.
    """
    xi = np.asarray(xi, dtype=np.float64)
    idx = basis_index(space, p)
    if subset is not None:
        idx = idx[np.asarray(subset, dtype=np.int64)]
    kinds = factor_kinds(space)
    nmax = max(orders(p)) + 1
    tab = {}
    for d in range(3):
        x = xi[:, d]
        tab[("chi", d)] = (poly1d.chi(nmax, x), poly1d.dchi(nmax, x))
        tab[("nu", d)] = (poly1d.nu(nmax, x), poly1d.dnu(nmax, x))
    Q = xi.shape[0]
    n = idx.shape[0]
    f = np.empty((3, Q, n))
    df = np.empty((3, Q, n))
    for d in range(3):
        for a in range(len(kinds)):
            sel = np.nonzero(idx[:, 0] == a)[0]
            if sel.size == 0:
                continue
            v, dv = tab[(kinds[a][d], d)]
            k = idx[sel, 1 + d]
            f[d][:, sel] = v[k].T
            df[d][:, sel] = dv[k].T
    val = f[0] * f[1] * f[2]
    grad = np.empty((Q, n, 3))
    grad[:, :, 0] = df[0] * f[1] * f[2]
    grad[:, :, 1] = f[0] * df[1] * f[2]
    grad[:, :, 2] = f[0] * f[1] * df[2]
    return idx[:, 0].copy(), val, grad
