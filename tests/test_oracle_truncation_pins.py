"""Pin of the oracle's finite-difference predictor by its truncation order.

For smooth fields that are not polynomials, the predictor of Eqs. 46-48
evaluated on the face lattice (Eq. 29 node values from the two cells'
centre values and gradients, central differences with lattice step h = c dt)
must approach the right-hand sides of Eqs. 46-48 evaluated exactly at the
face centre, here by symbolic differentiation of the fields.  With the cell
width and the lattice step both h, the node values carry O(h^2) errors, so
the predicted quantities differ from the exact right-hand sides by O(h^2):
the error falls by four when h halves.  A wrong stencil weight, sign or
index leaves an O(1) or O(h) remainder instead.

With all primitives linear the node values are exact and the remainder is
O(h^3); a wrong O(dt^2) coefficient would show there as order 2.

The TLBFS predictor (moment sums of the equilibria, Eqs. 30-32) and the
RTLBFS one (Eqs. 46-48) share the node values; Eqs. 44-45 make them differ
by the O(dt^3) remainder of the Taylor expansion only.
"""
import numpy as np
import pytest
import sympy as sp

from oracle import RTLBFS, TLBFS, OracleConfig, face_flux

CS2 = sp.Rational(1, 3)


def _fields(dim, linear=False):
    X = sp.symbols("x0:%d" % dim)
    if linear:
        # every primitive linear at once: Eq. 29 reproduces the node values
        # exactly, while the products rho u u and rho u T stay cubic
        c = [sp.Rational(k, 97) for k in (3, -5, 2, 7, -4, 6, 1, -3, 5, 2, -6, 4, 3, -2, 5, 1)]
        lin = lambda a0, i: a0 + sum(c[(i + j) % len(c)] * X[j] for j in range(dim))
        rho = lin(1, 0)
        u = [lin(sp.Rational(1, 25) * (a + 1), 3 * (a + 1)) / 4 for a in range(dim)]
        T = lin(sp.Rational(1, 2), 11)
        return X, rho, u, T
    if dim == 2:
        x, y = X
        rho = 1 + sp.Rational(1, 20) * sp.sin(x + sp.Rational(3, 10)) * sp.cos(sp.Rational(7, 10) * y + sp.Rational(1, 10))
        u = [sp.Rational(1, 25) * sp.sin(sp.Rational(4, 5) * x + sp.Rational(1, 2) * y + sp.Rational(1, 5)),
             sp.Rational(3, 100) * sp.cos(sp.Rational(3, 5) * x - sp.Rational(9, 10) * y + sp.Rational(2, 5))]
        T = sp.Rational(1, 2) + sp.Rational(1, 5) * sp.sin(sp.Rational(9, 10) * x + sp.Rational(2, 5) * y + sp.Rational(7, 10))
    else:
        x, y, z = X
        rho = 1 + sp.Rational(1, 20) * sp.sin(x + sp.Rational(3, 10) * z) * sp.cos(sp.Rational(7, 10) * y + sp.Rational(1, 10))
        u = [sp.Rational(1, 25) * sp.sin(sp.Rational(4, 5) * x + sp.Rational(1, 2) * y - sp.Rational(1, 5) * z),
             sp.Rational(3, 100) * sp.cos(sp.Rational(3, 5) * x - sp.Rational(9, 10) * y + sp.Rational(2, 5) * z),
             sp.Rational(1, 40) * sp.sin(sp.Rational(1, 2) * x + sp.Rational(3, 10) * y + sp.Rational(4, 5) * z + 1)]
        T = sp.Rational(1, 2) + sp.Rational(1, 5) * sp.sin(sp.Rational(9, 10) * x + sp.Rational(2, 5) * y + sp.Rational(3, 10) * z)
    return X, rho, u, T


def _exact_predictor(dim, linear=False):
    """Right-hand sides of Eqs. 46-48 (c_p = 1) as functions of (x, dt)."""
    X, rho, u, T = _fields(dim, linear)
    dt = sp.Symbol("dt")
    m = [rho * ua for ua in u]
    E = rho * T
    d = lambda f, a: sp.diff(f, X[a])
    Pi = [[rho * u[a] * u[b] + (CS2 * rho if a == b else 0) for b in range(dim)] for a in range(dim)]
    rho_s = rho - dt * sum(d(m[a], a) for a in range(dim)) \
        + dt ** 2 / 2 * sum(d(d(Pi[a][b], a), b) for a in range(dim) for b in range(dim))
    div_m = sum(d(m[g], g) for g in range(dim))
    m_s = [m[a] - dt * sum(d(Pi[a][b], b) for b in range(dim))
           + CS2 * dt ** 2 / 2 * sum(d(d(m[a], b) + d(m[b], a) + (div_m if a == b else 0), b) for b in range(dim))
           for a in range(dim)]
    E_s = E - dt * sum(d(E * u[a], a) for a in range(dim)) + CS2 * dt ** 2 / 2 * sum(d(d(E, a), a) for a in range(dim))
    exact = sp.lambdify([X, dt], [rho_s] + m_s + [E_s], "numpy")
    prims = sp.lambdify([X], [rho] + u + [T], "numpy")
    grads = sp.lambdify([X], [[d(f, a) for a in range(dim)] for f in [rho] + u + [T]], "numpy")
    return exact, prims, grads


def _predictor_errors(dim, axis, method, hs, linear=False):
    exact, prims, grads = _exact_predictor(dim, linear)
    xs = np.array([0.37, -0.21, 0.18][:dim])
    errs, preds = [], []
    for h in hs:
        xL, xR = xs.copy(), xs.copy()
        xL[axis] -= h / 2
        xR[axis] += h / 2
        cfg = OracleConfig(dim=dim, nu=0.05, chi=0.07, beta_g=0.0, gravity_axis=-1, dtl=h, method=method)
        _, pred = face_flux(cfg, axis, np.array(prims(xL)), np.array(grads(xL)), np.array(prims(xR)),
                            np.array(grads(xR)), h / 2, h / 2)
        ref = np.array(exact(xs, h), dtype=float)
        errs.append(np.abs(pred - ref).max())
        preds.append(pred)
    return np.array(errs), preds


@pytest.mark.parametrize("dim,axis", [(2, 0), (2, 1), (3, 0), (3, 2)])
def test_predictor_converges_to_eqs_46_48_at_second_order(dim, axis):
    hs = [0.2, 0.1, 0.05]
    errs, _ = _predictor_errors(dim, axis, RTLBFS, hs)
    orders = np.log2(errs[:-1] / errs[1:])
    # observed orders 2.0 within a few hundredths; the increments themselves are O(h)
    assert np.all((orders > 1.85) & (orders < 2.15)), (errs, orders)
    assert errs[-1] < 1e-4


@pytest.mark.parametrize("dim,axis", [(2, 0), (2, 1), (3, 1), (3, 2)])
def test_predictor_of_linear_fields_is_third_order(dim, axis):
    """Linear primitives: the node values are exact, so what remains is the
    central-difference error of the cubic products (dt * O(h^2)) and the
    dropped O(dt^3) Taylor term.  Any error in an O(dt^2) coefficient of
    Eqs. 46-48 (the 1/2, c_s^2, the three terms of Eq. 47) would leave an
    O(h^2) remainder and fail the order."""
    hs = [0.4, 0.2, 0.1]
    errs, _ = _predictor_errors(dim, axis, RTLBFS, hs, linear=True)
    orders = np.log2(errs[:-1] / errs[1:])
    assert np.all((orders > 2.8) & (orders < 3.2)), (errs, orders)


@pytest.mark.parametrize("dim", [2, 3])
def test_tlbfs_and_rtlbfs_predictors_differ_at_third_order(dim):
    hs = [0.2, 0.1, 0.05]
    _, pr = _predictor_errors(dim, 0, RTLBFS, hs)
    _, pt = _predictor_errors(dim, 0, TLBFS, hs)
    diffs = np.array([np.abs(a - b).max() for a, b in zip(pr, pt)])
    orders = np.log2(diffs[:-1] / diffs[1:])
    assert np.all((orders > 2.8) & (orders < 3.2)), (diffs, orders)
