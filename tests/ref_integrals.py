"""Reference integrals used to pin the oracle.  Independent of the oracle's code.

Everything here integrates the definition (Sec. 2, Eq. 2.1) directly, for unit
density and without the Coulomb constant:

    phi(P) = int dA / |P - Q|,        E(P) = int dA (P - Q) / |P - Q|^3.

* ``gl2``: the paper's reference method (Sec. 2): two nested 1-D Gauss-Legendre
  quadratures over the element (a triangle collapsed onto the unit square).
  Accurate to double precision for distance ratios above about 2.
* ``fan``: semi-analytic integration valid at any height.  The element is split
  into the triangles (F, V_k, V_k+1) around the foot F of P on the element's
  plane (signed areas); along each ray from F the integral is done in closed form,
  the remaining 1-D integral over the edge parameter by composite Gauss-Legendre.
* closed forms: the uniformly charged rectangle (textbook antiderivatives) and the
  in-plane potential of a convex polygon at an interior point.
"""
from __future__ import annotations

import math

import numpy as np


def leggauss01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def tri_vertices(g):
    g = np.asarray(g, float).ravel()
    return [g[0:3], g[3:6], g[6:9]]


def rect_vertices(g):
    g = np.asarray(g, float).ravel()
    P0, e1, e2 = g[0:3], g[3:6], g[6:9]
    return [P0, P0 + e1, P0 + e1 + e2, P0 + e2]


def polygon(kind, g):
    return tri_vertices(g) if kind == 0 else rect_vertices(g)


# ---------------------------------------------------------------- GL2 -----
def gl2(kind, g, P, n=32):
    """(phi, Ex, Ey, Ez) by nested Gauss-Legendre quadrature."""
    P = np.asarray(P, float)
    x, w = leggauss01(n)
    U, V = np.meshgrid(x, x, indexing="ij")
    WU, WV = np.meshgrid(w, w, indexing="ij")
    g = np.asarray(g, float).ravel()
    if kind == 0:
        A, B, C = g[0:3], g[3:6], g[6:9]
        # Q = A + u (B - A) + u v (C - B),  dA = 2 area u du dv
        Q = A + U[..., None] * (B - A) + (U * V)[..., None] * (C - B)
        jac = np.linalg.norm(np.cross(B - A, C - A)) * U
    else:
        P0, e1, e2 = g[0:3], g[3:6], g[6:9]
        Q = P0 + U[..., None] * e1 + V[..., None] * e2
        jac = np.linalg.norm(e1) * np.linalg.norm(e2) * np.ones_like(U)
    d = P - Q
    r = np.linalg.norm(d, axis=-1)
    wt = WU * WV * jac
    phi = np.sum(wt / r)
    E = np.sum((wt / r ** 3)[..., None] * d, axis=(0, 1))
    return np.array([phi, E[0], E[1], E[2]])


# ---------------------------------------------------------------- fan -----
def fan(kind, g, P, n_sub=24, n_gl=24):
    """(phi, Ex, Ey, Ez) semi-analytically; P must not lie in the element's plane
    outside the element (h = 0 is allowed only for the potential)."""
    P = np.asarray(P, float)
    V = polygon(kind, g)
    nrm = np.cross(V[1] - V[0], V[2] - V[0])
    nrm /= np.linalg.norm(nrm)
    h = float(np.dot(P - V[0], nrm))
    F = P - h * nrm
    ah = abs(h)
    x, w = leggauss01(n_gl)
    # composite rule on [0, 1]
    edges = np.linspace(0.0, 1.0, n_sub + 1)
    vv = (edges[:-1, None] + (edges[1:] - edges[:-1])[:, None] * x[None, :]).ravel()
    ww = ((edges[1:] - edges[:-1])[:, None] * w[None, :]).ravel()
    phi = 0.0
    E = np.zeros(3)
    for k in range(len(V)):
        Va, Vb = V[k], V[(k + 1) % len(V)]
        R0 = Va - F
        dv = Vb - Va
        twoA = float(np.dot(np.cross(R0, dv), nrm))  # signed
        if twoA == 0.0:
            continue
        R = R0[None, :] + vv[:, None] * dv[None, :]
        c = np.linalg.norm(R, axis=1)
        s = np.sqrt(h * h + c * c)
        # int_0^1 u du / sqrt(h^2 + u^2 c^2) = 1 / (s + |h|)
        phi += twoA * np.sum(ww / (s + ah))
        # normal part: h int_0^1 u du / (h^2 + u^2 c^2)^1.5 = sign(h) / (s (s + |h|))
        if h != 0.0:
            E += twoA * math.copysign(1.0, h) * np.sum(ww / (s * (s + ah))) * nrm
            # in-plane: -R int_0^1 u^2 du / (...)^1.5 = -R (asinh(c/|h|) - c/s) / c^3
            f = (np.arcsinh(c / ah) - c / s) / c ** 3
            E -= twoA * np.sum((ww * f)[:, None] * R, axis=0)
    return np.array([phi, E[0], E[1], E[2]])


# ------------------------------------------------------- closed forms -----
def rect_closed_form(g, P):
    """Uniformly charged rectangle (orthogonal sides): potential and field, textbook
    antiderivatives in the rectangle's own frame."""
    g = np.asarray(g, float).ravel()
    P0, e1, e2 = g[0:3], g[3:6], g[6:9]
    a, b = np.linalg.norm(e1), np.linalg.norm(e2)
    ux, uy = e1 / a, e2 / b
    uz = np.cross(ux, uy)
    d = np.asarray(P, float) - P0
    x0, y0, z = np.dot(d, ux), np.dot(d, uy), np.dot(d, uz)
    if abs(z) < 1e-13 * max(a, b):
        z = 0.0  # in the plane: principal value, no normal field

    def F(X, Y):  # antiderivative of 1/R over x and y, X = x - x0, Y = y - y0
        R = math.sqrt(X * X + Y * Y + z * z)
        t = 0.0
        rx = math.hypot(X, z)
        ry = math.hypot(Y, z)
        if rx > 0:
            t += X * math.asinh(Y / rx)
        if ry > 0:
            t += Y * math.asinh(X / ry)
        if z != 0:
            t -= z * math.atan(X * Y / (z * R))
        return t

    def Gz(X, Y):
        R = math.sqrt(X * X + Y * Y + z * z)
        return math.atan(X * Y / (z * R)) if z != 0 else 0.0

    def Gx(X, Y):  # antiderivative of -X/R^3 dX dY -> asinh(Y / hypot(X, z))
        rx = math.hypot(X, z)
        return math.asinh(Y / rx)

    def Gy(X, Y):
        ry = math.hypot(Y, z)
        return math.asinh(X / ry)

    X1, X2, Y1, Y2 = -x0, a - x0, -y0, b - y0

    def box(fn):
        return fn(X2, Y2) - fn(X1, Y2) - fn(X2, Y1) + fn(X1, Y1)

    phi = box(F)
    Ez = box(Gz) if z != 0 else 0.0
    # E_x = int int (x0 - x)/R^3 = [asinh(Y/hypot(X,z))] with X from X1 to X2 ... sign below
    Ex = (Gx(X2, Y2) - Gx(X2, Y1)) - (Gx(X1, Y2) - Gx(X1, Y1))
    Ey = (Gy(X2, Y2) - Gy(X1, Y2)) - (Gy(X2, Y1) - Gy(X1, Y1))
    Evec = Ex * ux + Ey * uy + Ez * uz
    return np.array([phi, Evec[0], Evec[1], Evec[2]])


def rect_gradient_closed_form(g, P):
    """Field gradient G_ij = dE_i/dP_j = -d^2 phi/dP_i dP_j of the uniformly charged
    rectangle (orthogonal sides), P off the rectangle's plane.  In the rectangle's frame,
    with X = x - x0, Y = y - y0, R = sqrt(X^2 + Y^2 + z^2) and corner sums
    C[f] = f(X2, Y2) - f(X1, Y2) - f(X2, Y1) + f(X1, Y1), the Hessian of phi is
        H_xx = -C[X Y / ((X^2 + z^2) R)],  H_yy = -C[X Y / ((Y^2 + z^2) R)],
        H_xy = C[1 / R],  H_xz = C[z Y / ((X^2 + z^2) R)],  H_yz = C[z X / ((Y^2 + z^2) R)],
        H_zz = -(H_xx + H_yy)   (Laplace),
    using int dY / R^3 = Y / ((X^2 + z^2) R).  Returns the 3x3 matrix in global axes."""
    g = np.asarray(g, float).ravel()
    P0, e1, e2 = g[0:3], g[3:6], g[6:9]
    a, b = np.linalg.norm(e1), np.linalg.norm(e2)
    ux, uy = e1 / a, e2 / b
    uz = np.cross(ux, uy)
    d = np.asarray(P, float) - P0
    x0, y0, z = np.dot(d, ux), np.dot(d, uy), np.dot(d, uz)
    if z == 0.0:
        raise ValueError("point in the rectangle's plane")
    X1, X2, Y1, Y2 = -x0, a - x0, -y0, b - y0

    def C(fn):
        return fn(X2, Y2) - fn(X1, Y2) - fn(X2, Y1) + fn(X1, Y1)

    def R(X, Y):
        return math.sqrt(X * X + Y * Y + z * z)

    Hxx = -C(lambda X, Y: X * Y / ((X * X + z * z) * R(X, Y)))
    Hyy = -C(lambda X, Y: X * Y / ((Y * Y + z * z) * R(X, Y)))
    Hxy = C(lambda X, Y: 1.0 / R(X, Y))
    Hxz = C(lambda X, Y: z * Y / ((X * X + z * z) * R(X, Y)))
    Hyz = C(lambda X, Y: z * X / ((Y * Y + z * z) * R(X, Y)))
    H = np.array([[Hxx, Hxy, Hxz], [Hxy, Hyy, Hyz], [Hxz, Hyz, -(Hxx + Hyy)]])
    U = np.stack([ux, uy, uz], axis=1)  # local -> global
    return -(U @ H @ U.T)


def gl2_gradient(kind, g, P, n=48):
    """Field gradient by nested Gauss-Legendre quadrature of the kernel
    (3 d d^T - r^2 I) / r^5 ... with the sign of dE/dP: (r^2 I - 3 d d^T) / r^5."""
    P = np.asarray(P, float)
    x, w = leggauss01(n)
    U, V = np.meshgrid(x, x, indexing="ij")
    WU, WV = np.meshgrid(w, w, indexing="ij")
    g = np.asarray(g, float).ravel()
    if kind == 0:
        A, B, Cc = g[0:3], g[3:6], g[6:9]
        Q = A + U[..., None] * (B - A) + (U * V)[..., None] * (Cc - B)
        jac = np.linalg.norm(np.cross(B - A, Cc - A)) * U
    else:
        P0, e1, e2 = g[0:3], g[3:6], g[6:9]
        Q = P0 + U[..., None] * e1 + V[..., None] * e2
        jac = np.linalg.norm(e1) * np.linalg.norm(e2) * np.ones_like(U)
    d = (P - Q).reshape(-1, 3)
    r2 = np.sum(d * d, axis=1)
    wt = (WU * WV * jac).ravel() / r2 ** 2.5
    return np.einsum("k,k->", wt, r2) * np.eye(3) - 3.0 * np.einsum("k,ki,kj->ij", wt, d, d)


def gradient_6(G):
    """3x3 -> (xx, yy, zz, xy, xz, yz)."""
    return np.array([G[0, 0], G[1, 1], G[2, 2], G[0, 1], G[0, 2], G[1, 2]])


def polygon_inplane_potential(V, P):
    """int dA / |Q - P| for P inside a convex planar polygon V (in plane):
    sum over edges of h_e [asinh(t2 / h_e) - asinh(t1 / h_e)]."""
    P = np.asarray(P, float)
    tot = 0.0
    for k in range(len(V)):
        A, B = np.asarray(V[k], float), np.asarray(V[(k + 1) % len(V)], float)
        t = B - A
        L = np.linalg.norm(t)
        t /= L
        t1 = float(np.dot(A - P, t))
        t2 = float(np.dot(B - P, t))
        foot = A - t1 * t
        h = float(np.linalg.norm(foot - P))
        if h > 0:
            tot += h * (math.asinh(t2 / h) - math.asinh(t1 / h))
    return tot


def rel_err_phi(a, ref):
    return abs(a[0] - ref[0]) / abs(ref[0])


def rel_err_E(a, ref):
    """Sec. 2: sum over components of |E_j - E_j,ref| / |E_ref|."""
    return float(np.sum(np.abs(np.asarray(a[1:4]) - np.asarray(ref[1:4]))) / np.linalg.norm(ref[1:4]))
