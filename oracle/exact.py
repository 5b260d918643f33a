"""Exact solution of one implicit HDG stage on small periodic squares (oracle).

Test infrastructure: only tests and their fixture scripts use this module.

The stage system is the HDG upwind form (Eq. bilinear_HDG_upwind with the
flux condition, one stage of Eq. general_linear_system with alpha = 1) in
the symmetric variables phi = h sqrt(g/H), kappa = sqrt(g H) dt, phi_B = 1
and the stabilisation written per side as tau: for every cell K and every
test function

    (phi, psi)_K - kappa (u, grad psi)_K + kappa <u.n + tau (phi - lam), psi>_dK = (r_phi, psi)_K
    (u, w)_K + dt f (k x u, w)_K - kappa (phi, div w)_K + kappa <lam, w.n>_dK  = (r_u, w)_K

and on every facet e, for every trace test function mu,

    sum over the two cells K of e of  <u_K.n_K + tau (phi_K - lam), mu>_e = 0.

Everything here is computed in exact arithmetic: the mesh coordinates, dt,
g, H, f, tau and the right-hand side coefficients are rationals (with g H
and g / H perfect squares, so that kappa and sqrt(g/H) are rational), and the
only irrational number that enters is the length sqrt(2) of the diagonal
facets, so the whole system lives in Q(sqrt 2) and is solved there by exact
LU (sympy's DomainMatrix over the algebraic field).  Nothing is shared with
the floating-point oracle: the basis is Silvester's closed-form Lagrange
polynomial on the equispaced lattice written in barycentric coordinates,
integrals use the exact monomial moments of the reference triangle
(int xi^a eta^b = a! b! / (a + b + 2)!) and of the unit interval, and facets
are identified by their midpoints modulo the period.

Conventions (the documented data format, which the library and the oracle
follow as well): DG nodes at the lattice (i/p, j/p), j-major then i, on the
reference triangle mapped to x = a + xi (b - a) + eta (c - a); local facet i
of a cell runs from corner (i+1)%3 to (i+2)%3; facets are numbered by first
appearance scanning cells and local facets in order; the first cell fixes the
facet's direction and trace node k sits at parameter k/p along it.
"""
from __future__ import annotations

from fractions import Fraction
from math import factorial

import sympy as sp
from sympy.polys.matrices import DomainMatrix

X, Y = sp.symbols("x y")
S = sp.symbols("s")          # parameter along a facet
XI, ETA = sp.symbols("xi eta")


def _rat(v):
    """Exact rational of an int, a Fraction, a sympy number or a float (the float's
    own binary value, so inputs stored as doubles are taken exactly)."""
    if isinstance(v, sp.Basic):
        return v
    return sp.Rational(Fraction(v))


def lattice(p):
    """Lattice indices (i, j), j-major then i; node (i/p, j/p)."""
    return [(i, j) for j in range(p + 1) for i in range(p + 1 - j)]


def silvester(p, i, j, la, lb, lc):
    """Lagrange polynomial of lattice node (i, j) in barycentric coordinates
    (la, lb, lc) of corners (a, b, c): the node has barycentric indices
    (p - i - j, i, j) and the polynomial is the product over each coordinate of
    prod_{s < index} (p l - s) / (index - s)."""
    out = sp.Integer(1)
    for lam, idx in ((la, p - i - j), (lb, i), (lc, j)):
        for s in range(idx):
            out *= (p * lam - s) / sp.Integer(idx - s)
    return sp.expand(out)


def lagrange_1d(p, k, s):
    """Lagrange polynomial of node k/p on [0, 1]."""
    out = sp.Integer(1)
    for q in range(p + 1):
        if q != k:
            out *= (s - sp.Rational(q, p)) / (sp.Rational(k, p) - sp.Rational(q, p))
    return sp.expand(out)


def _ref_moment(a, b):
    """int over the reference triangle of xi^a eta^b."""
    return sp.Rational(factorial(a) * factorial(b), factorial(a + b + 2))


def _powers(base, k):
    out = [sp.Poly(1, *base.gens, domain=sp.QQ)]
    for _ in range(k):
        out.append(out[-1] * base)
    return out


def substitute(poly_xy, xs, ys):
    """poly(x, y) with x, y replaced by the polynomials xs, ys (same generators)."""
    deg = max(poly_xy.total_degree(), 0)
    px, py = _powers(xs, deg), _powers(ys, deg)
    out = sp.Poly(0, *xs.gens, domain=sp.QQ)
    for (a, b), c in poly_xy.terms():
        out += px[a] * py[b] * c
    return out


def integrate_cell(poly_xy, corners):
    """Exact integral of a polynomial in (x, y) over the triangle with the given corners."""
    (ax, ay), (bx, by), (cx, cy) = corners
    jac = (bx - ax) * (cy - ay) - (by - ay) * (cx - ax)     # = 2 |K| (counter-clockwise)
    xs = sp.Poly(ax + XI * (bx - ax) + ETA * (cx - ax), XI, ETA, domain=sp.QQ)
    ys = sp.Poly(ay + XI * (by - ay) + ETA * (cy - ay), XI, ETA, domain=sp.QQ)
    ref = substitute(poly_xy, xs, ys)
    return jac * sum((c * _ref_moment(a, b) for (a, b), c in ref.terms()), sp.Integer(0))


def integrate_segment(poly_s, length):
    """Exact integral over a straight facet of a polynomial in its parameter s in [0, 1]."""
    return length * sum((c / sp.Integer(a + 1) for (a,), c in poly_s.terms()), sp.Integer(0))


class ExactStage:
    """The stage system on a periodic n x n square (cells split along (0,0)-(1,1),
    the torus generator's convention), assembled and solved over Q(sqrt 2)."""

    def __init__(self, cells, p, dt, g, H, f, tau=1, period=1):
        """cells: list of 3 unwrapped corners (x, y) per cell, counter-clockwise, rationals."""
        self.p, self.m = p, p + 1
        self.n = (p + 1) * (p + 2) // 2
        self.cells = [[(_rat(a), _rat(b)) for (a, b) in c] for c in cells]
        self.dt, self.g, self.H, self.f, self.tau = map(_rat, (dt, g, H, f, tau))
        self.period = _rat(period)
        c = sp.sqrt(self.g * self.H)
        hs = sp.sqrt(self.g / self.H)
        if not (c.is_Rational and hs.is_Rational):
            raise ValueError("g H and g / H must be squares of rationals")
        self.kappa, self.hscale = c * self.dt, hs
        self._facets()
        self._basis()

    # -- topology: facets keyed by their midpoint modulo the period
    def _facets(self):
        self.facets = []          # (start, end) of the owner's traversal
        self.cell_facet = []      # per cell, per local facet: (facet id, same direction?)
        key_of = {}
        for K, cor in enumerate(self.cells):
            row = []
            for i in range(3):
                A, B = cor[(i + 1) % 3], cor[(i + 2) % 3]
                mid = tuple(((A[d] + B[d]) / 2) % self.period for d in range(2))
                if mid not in key_of:
                    key_of[mid] = len(self.facets)
                    self.facets.append((A, B))
                    row.append((key_of[mid], True))
                else:
                    e = key_of[mid]
                    S0, E0 = self.facets[e]
                    dA = (B[0] - A[0], B[1] - A[1])
                    dE = (E0[0] - S0[0], E0[1] - S0[1])
                    if dA == dE:
                        same = True
                    elif dA == (-dE[0], -dE[1]):
                        same = False
                    else:
                        raise ValueError("facet key collision")
                    row.append((e, same))
            self.cell_facet.append(row)
        self.ne = len(self.facets)

    # -- basis functions on each cell, as polynomials in (x, y)
    def _basis(self):
        self.phi = []
        for cor in self.cells:
            (ax, ay), (bx, by), (cx, cy) = cor
            det = (bx - ax) * (cy - ay) - (by - ay) * (cx - ax)
            xi = ((cy - ay) * (X - ax) - (cx - ax) * (Y - ay)) / det
            eta = (-(by - ay) * (X - ax) + (bx - ax) * (Y - ay)) / det
            lb, lc = sp.expand(xi), sp.expand(eta)
            la = sp.expand(1 - lb - lc)
            self.phi.append([sp.Poly(silvester(self.p, i, j, la, lb, lc), X, Y, domain=sp.QQ)
                             for (i, j) in lattice(self.p)])

    # -- unknown numbering: cell K field fd node i, then facet e node k
    def cidx(self, K, fd, i):
        return (K * 3 + fd) * self.n + i

    def tidx(self, e, k):
        return len(self.cells) * 3 * self.n + e * self.m + k

    def system(self, r_cell):
        """Matrix and right-hand side (lists of sympy numbers).  r_cell[K][fd][i]:
        rational DG coefficients of (r_h, r_u1, r_u2)."""
        p, n, m = self.p, self.n, self.m
        kap, tau, dt, f = self.kappa, self.tau, self.dt, self.f
        N = len(self.cells) * 3 * n + self.ne * m
        A = {}
        rhs = [sp.Integer(0)] * N

        def add(r, c, v):
            if v != 0:
                A[(r, c)] = sp.expand(A.get((r, c), 0) + v)

        mu = [sp.Poly(lagrange_1d(p, k, S), S, domain=sp.QQ) for k in range(m)]
        for K, cor in enumerate(self.cells):
            ph = self.phi[K]
            dx = [b.diff(X) for b in ph]
            dy = [b.diff(Y) for b in ph]
            mass = [[integrate_cell(ph[i] * ph[j], cor) for j in range(n)] for i in range(n)]
            # (phi_j, d psi_i): gradient of the test function
            gx = [[integrate_cell(ph[j] * dx[i], cor) for j in range(n)] for i in range(n)]
            gy = [[integrate_cell(ph[j] * dy[i], cor) for j in range(n)] for i in range(n)]
            for i in range(n):
                for j in range(n):
                    # phi row
                    add(self.cidx(K, 0, i), self.cidx(K, 0, j), mass[i][j])
                    add(self.cidx(K, 0, i), self.cidx(K, 1, j), -kap * gx[i][j])
                    add(self.cidx(K, 0, i), self.cidx(K, 2, j), -kap * gy[i][j])
                    # u rows: (u, w) + dt f (k x u, w) - kappa (phi, div w); k x u = (-u2, u1)
                    add(self.cidx(K, 1, i), self.cidx(K, 1, j), mass[i][j])
                    add(self.cidx(K, 1, i), self.cidx(K, 2, j), -dt * f * mass[i][j])
                    add(self.cidx(K, 1, i), self.cidx(K, 0, j), -kap * gx[i][j])
                    add(self.cidx(K, 2, i), self.cidx(K, 2, j), mass[i][j])
                    add(self.cidx(K, 2, i), self.cidx(K, 1, j), dt * f * mass[i][j])
                    add(self.cidx(K, 2, i), self.cidx(K, 0, j), -kap * gy[i][j])
                    # right-hand sides (r_phi = sqrt(g/H) r_h)
                    rhs[self.cidx(K, 0, i)] += mass[i][j] * self.hscale * _rat(r_cell[K][0][j])
                    rhs[self.cidx(K, 1, i)] += mass[i][j] * _rat(r_cell[K][1][j])
                    rhs[self.cidx(K, 2, i)] += mass[i][j] * _rat(r_cell[K][2][j])
            for loc in range(3):
                Apt, Bpt = cor[(loc + 1) % 3], cor[(loc + 2) % 3]
                tx, ty = Bpt[0] - Apt[0], Bpt[1] - Apt[1]
                length = sp.sqrt(tx * tx + ty * ty)
                nx, ny = ty / length, -tx / length          # outward for a counter-clockwise cell
                xs = sp.Poly(Apt[0] + S * tx, S, domain=sp.QQ)
                ys = sp.Poly(Apt[1] + S * ty, S, domain=sp.QQ)
                pv = [substitute(b, xs, ys) for b in ph]
                e, same = self.cell_facet[K][loc]
                # trace basis in this cell's parameter: s along the facet direction or reversed
                rev = sp.Poly(1 - S, S, domain=sp.QQ)
                mu_c = mu if same else [mk.compose(rev) for mk in mu]
                pp = [[integrate_segment(pv[i] * pv[j], length) for j in range(n)] for i in range(n)]
                pm = [[integrate_segment(pv[i] * mu_c[k], length) for k in range(m)] for i in range(n)]
                for i in range(n):
                    for j in range(n):
                        # kappa <u.n + tau phi, psi>
                        add(self.cidx(K, 0, i), self.cidx(K, 0, j), kap * tau * pp[i][j])
                        add(self.cidx(K, 0, i), self.cidx(K, 1, j), kap * nx * pp[i][j])
                        add(self.cidx(K, 0, i), self.cidx(K, 2, j), kap * ny * pp[i][j])
                    for k in range(m):
                        add(self.cidx(K, 0, i), self.tidx(e, k), -kap * tau * pm[i][k])   # -kappa tau <lam, psi>
                        add(self.cidx(K, 1, i), self.tidx(e, k), kap * nx * pm[i][k])     # kappa <lam, w.n>
                        add(self.cidx(K, 2, i), self.tidx(e, k), kap * ny * pm[i][k])
                # flux condition rows of facet e: <u.n + tau (phi - lam), mu_k>
                mm = [[integrate_segment(mu_c[k] * mu_c[l], length) for l in range(m)] for k in range(m)]
                for k in range(m):
                    for j in range(n):
                        add(self.tidx(e, k), self.cidx(K, 0, j), tau * pm[j][k])
                        add(self.tidx(e, k), self.cidx(K, 1, j), nx * pm[j][k])
                        add(self.tidx(e, k), self.cidx(K, 2, j), ny * pm[j][k])
                    for l in range(m):
                        add(self.tidx(e, k), self.tidx(e, l), -tau * mm[k][l])
        return N, A, rhs

    def solve(self, r_cell):
        """Exact (h, u1, u2) coefficients per cell and trace values per facet node,
        as sympy numbers in Q(sqrt 2)."""
        N, A, rhs = self.system(r_cell)
        K = sp.QQ.algebraic_field(sp.sqrt(2))
        dense = [[K.from_sympy(sp.sympify(A.get((i, j), 0))) for j in range(N)] for i in range(N)]
        b = [[K.from_sympy(sp.sympify(v))] for v in rhs]
        M = DomainMatrix(dense, (N, N), K)
        sol = M.lu_solve(DomainMatrix(b, (N, 1), K)).to_Matrix()
        x = [sol[i, 0] for i in range(N)]
        q = [[[x[self.cidx(Kc, fd, i)] / (self.hscale if fd == 0 else 1) for i in range(self.n)]
              for fd in range(3)] for Kc in range(len(self.cells))]
        lam = [[x[self.tidx(e, k)] for k in range(self.m)] for e in range(self.ne)]
        return q, lam


def torus_cells(nsq, period=1):
    """Cells of the n x n periodic square split along (0,0)-(1,1): per square the
    lower-right triangle (00, 10, 11) then the upper-left one (00, 11, 01),
    squares in row-major order (j outer), unwrapped corners."""
    h = sp.Rational(period, nsq)
    out = []
    for j in range(nsq):
        for i in range(nsq):
            c = {"00": (i * h, j * h), "10": ((i + 1) * h, j * h), "11": ((i + 1) * h, (j + 1) * h),
                 "01": (i * h, (j + 1) * h)}
            out.append([c["00"], c["10"], c["11"]])
            out.append([c["00"], c["11"], c["01"]])
    return out


def to_float(v, digits=30):
    return float(sp.N(v, digits))
