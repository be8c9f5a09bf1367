"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each ``pin_*`` takes an ``oracle.Oracle`` and raises AssertionError when the oracle disagrees
with the fact it is checked against.  None of them re-types the oracle's formulas: the
references are the literal double sum of Eq. (1), finite differences of that sum, textbook
Laplacian closed forms at p = 2 (via scipy), hand-worked small graphs, and invariants that
Eq. (1) implies.  ``tests/test_oracle_mutants.py`` runs the whole battery against deliberately
broken builds of the oracle to show that each plausible mistake is caught.
"""
from __future__ import annotations

import numpy as np

import oracle as orc

P_LEVELS = (2.0, 1.6, 1.3, 1.1, 1.05)


def csr_from_dense(W):
    W = np.asarray(W, dtype=np.float64)
    n = W.shape[0]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    cols, vals = [], []
    for i in range(n):
        nz = np.nonzero(W[i])[0]
        cols.extend(nz.tolist())
        vals.extend(W[i, nz].tolist())
        rowptr[i + 1] = len(cols)
    return rowptr, np.array(cols, dtype=np.int32), np.array(vals, dtype=np.float64)


def random_sym_weights(n, density, rng, lo=0.2, hi=1.7):
    A = np.triu(rng.uniform(lo, hi, size=(n, n)) * (rng.random((n, n)) < density), k=1)
    return A + A.T


def spread_block(n, k, rng):
    """Columns that are shuffled, jittered, evenly spaced values: no near-ties, no entry near 0."""
    base = np.linspace(-2.0, 2.0, n)
    base = np.where(np.abs(base) < 0.2, np.sign(base + 1e-9) * 0.3, base)
    cols = []
    for _ in range(k):
        cols.append(rng.permutation(base) + rng.uniform(-0.05, 0.05, n))
    return np.stack(cols, axis=1)


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# --- worked examples -------------------------------------------------------------------------

def pin_two_node(o):
    """One edge of weight w: F = w|a-b|^p / (|a|^p + |b|^p) (Eq. (1) with both ordered pairs);
    at u = (1, -1) F = w 2^(p-1) and u is a critical point."""
    w = 0.7
    rowptr = np.array([0, 1, 2], dtype=np.int64)
    col = np.array([1, 0], dtype=np.int32)
    wt = np.array([w, w])
    a, b = 0.3, -1.1
    U = np.array([[a, 1.0], [b, -1.0]])
    for p in P_LEVELS:
        F, Fc, N, D = o.objective(rowptr, col, wt, U, p)
        assert abs(Fc[0] - w * abs(a - b) ** p / (abs(a) ** p + abs(b) ** p)) < 1e-14
        assert abs(Fc[1] - w * 2.0 ** (p - 1.0)) < 1e-14
        assert abs(N[1] - w * 2.0 ** p) < 1e-14 and abs(D[1] - 2.0) < 1e-14
        G, _ = o.grad(rowptr, col, wt, U, p)
        assert np.max(np.abs(G[:, 1])) < 1e-14

        # gradient of the closed form, by central differences
        def f(x, y):
            return w * abs(x - y) ** p / (abs(x) ** p + abs(y) ** p)

        h = 1e-6
        ga = (f(a + h, b) - f(a - h, b)) / (2 * h)
        gb = (f(a, b + h) - f(a, b - h)) / (2 * h)
        assert abs(G[0, 0] - ga) < 1e-8 and abs(G[1, 0] - gb) < 1e-8


def pin_three_path(o):
    """Path 0-1-2 with unit weights and u = (1, 0, -1): N = 2, D = 2, F = 1 and G = 0 for every p
    (the two edges carry |x| = 1; Delta_p u = (1, 0, -1) = phi_p(u))."""
    rowptr = np.array([0, 1, 3, 4], dtype=np.int64)
    col = np.array([1, 0, 2, 1], dtype=np.int32)
    wt = np.ones(4)
    U = np.array([[1.0], [0.0], [-1.0]])
    for p in P_LEVELS:
        F, Fc, N, D = o.objective(rowptr, col, wt, U, p)
        assert abs(F - 1.0) < 1e-15 and abs(N[0] - 2.0) < 1e-15 and abs(D[0] - 2.0) < 1e-15
        L = o.plap(rowptr, col, wt, U, p)
        assert np.max(np.abs(L[:, 0] - np.array([1.0, 0.0, -1.0]))) < 1e-15
        G, _ = o.grad(rowptr, col, wt, U, p)
        assert np.max(np.abs(G)) < 1e-15


# --- brute force and finite differences of Eq. (1) -------------------------------------------

def pin_brute_force(o):
    """Oracle F equals the literal ordered-pair double sum of Eq. (1) on small dense graphs."""
    rng = np.random.default_rng(11)
    for trial in range(3):
        n, k = 9 + trial, 2 + trial
        W = random_sym_weights(n, 0.5, rng)
        U = rng.standard_normal((n, k))
        rp, c, w = csr_from_dense(W)
        for p in P_LEVELS:
            F, Fc, _, _ = o.objective(rp, c, w, U, p)
            ref = orc.brute_objective(W, U, p)
            assert abs(F - ref) <= 1e-12 * abs(ref), (trial, p, F, ref)
            for l in range(k):
                refl = orc.brute_objective(W, U[:, l:l + 1], p)
                assert abs(Fc[l] - refl) <= 1e-12 * abs(refl)


def pin_grad_fd(o):
    """Oracle gradient equals central differences of the brute-force F."""
    rng = np.random.default_rng(12)
    n, k = 8, 2
    W = random_sym_weights(n, 0.6, rng)
    rp, c, w = csr_from_dense(W)
    U = spread_block(n, k, rng)
    h = 1e-6
    for p in P_LEVELS:
        G, _ = o.grad(rp, c, w, U, p)
        Gfd = np.zeros_like(U)
        for i in range(n):
            for l in range(k):
                Up = U.copy()
                Up[i, l] += h
                Um = U.copy()
                Um[i, l] -= h
                Gfd[i, l] = (orc.brute_objective(W, Up, p) - orc.brute_objective(W, Um, p)) / (2 * h)
        assert _rel(G, Gfd) < 1e-7, (p, _rel(G, Gfd))


def pin_hvp_fd(o):
    """Oracle H v equals mixed second differences of the brute-force F, entry by entry, and
    <v, H v> equals the second difference of F along v."""
    rng = np.random.default_rng(13)
    n, k = 7, 2
    W = random_sym_weights(n, 0.7, rng)
    rp, c, w = csr_from_dense(W)
    U = spread_block(n, k, rng)
    V = rng.standard_normal((n, k))
    h = 1e-4
    for p in P_LEVELS:
        HV, _, _ = o.hvp(rp, c, w, U, V, p, 1e-12)
        F = lambda X: orc.brute_objective(W, X, p)  # noqa: E731
        ref = np.zeros_like(U)
        for i in range(n):
            for l in range(k):
                E = np.zeros_like(U)
                E[i, l] = h
                ref[i, l] = (F(U + h * V + E) - F(U + h * V - E) - F(U - h * V + E) + F(U - h * V - E)) / (4 * h * h)
        assert _rel(HV, ref) < 1e-5, (p, _rel(HV, ref))
        quad = (F(U + h * V) - 2 * F(U) + F(U - h * V)) / (h * h)
        assert abs(np.sum(V * HV) - quad) <= 1e-5 * max(abs(quad), 1.0), (p, np.sum(V * HV), quad)


def pin_algorithm1_form(o):
    """Assemble each column's Hessian H^l from the oracle's products with unit vectors; it is
    symmetric and Algorithm 1's r = D[l] * eta - (diag(H^l) - H^l) eta reproduces the oracle's
    product with an arbitrary eta."""
    rng = np.random.default_rng(14)
    n, k = 10, 2
    W = random_sym_weights(n, 0.5, rng)
    rp, c, w = csr_from_dense(W)
    U = spread_block(n, k, rng)
    eta = rng.standard_normal((n, k))
    for p in P_LEVELS:
        H = np.zeros((k, n, n))
        for j in range(n):
            E = np.zeros((n, k))
            E[j, :] = 1.0
            HV, _, _ = o.hvp(rp, c, w, U, E, p, 1e-12)
            H[:, :, j] = HV.T
        HVe, _, _ = o.hvp(rp, c, w, U, eta, p, 1e-12)
        for l in range(k):
            Hl = H[l]
            assert np.max(np.abs(Hl - Hl.T)) <= 1e-10 * np.max(np.abs(Hl))
            Dl = np.diag(Hl)
            Hbar = np.diag(Dl) - Hl
            r = Dl * eta[:, l] - Hbar @ eta[:, l]
            assert _rel(r, HVe[:, l]) < 1e-12


def pin_hvp_sparse(o):
    """Algorithm 1 read with sparse D[l], H[l]: the sparse Hessian part is (p/D) d/dt [Delta_p(u + t v)
    - F phi_p(u + t v)] at t = 0 with D, F fixed, checked by central differences of the oracle's
    p-Laplacian (pinned above) and of phi_p; assembled per column it is symmetric and zero off the
    graph's pattern and diagonal; the exact operator minus it is -(p/D)(g a + phi b) with a = phi^T v,
    b = g^T v (the rank-2 term)."""
    rng = np.random.default_rng(21)
    n, k = 12, 2
    W = random_sym_weights(n, 0.4, rng)
    rp, c, w = csr_from_dense(W)
    U = spread_block(n, k, rng)
    V = rng.standard_normal((n, k))
    h = 1e-6
    for p in (1.6, 1.3):
        HVs = o.hvp_sparse(rp, c, w, U, V, p, 1e-12)
        _, Fc, _, D = o.objective(rp, c, w, U, p)
        phi = lambda X: np.sign(X) * np.abs(X) ** (p - 1)  # noqa: E731
        Lp = o.plap(rp, c, w, U + h * V, p)
        Lm = o.plap(rp, c, w, U - h * V, p)
        fd = (p / D) * ((Lp - Lm) / (2 * h) - Fc * (phi(U + h * V) - phi(U - h * V)) / (2 * h))
        assert np.max(np.abs(HVs - fd)) <= 1e-6 * np.max(np.abs(fd))
        H = np.zeros((k, n, n))
        for j in range(n):
            E = np.zeros((n, k))
            E[j, :] = 1.0
            H[:, :, j] = o.hvp_sparse(rp, c, w, U, E, p, 1e-12).T
        off = (W == 0) & ~np.eye(n, dtype=bool)
        for l in range(k):
            assert np.all(H[l][off] == 0.0)
            assert np.max(np.abs(H[l] - H[l].T)) <= 1e-12 * np.max(np.abs(H[l]))
        HV, G, _ = o.hvp(rp, c, w, U, V, p, 1e-12)
        a = np.sum(phi(U) * V, axis=0)
        b = np.sum(G * V, axis=0)
        assert np.allclose(HV - HVs, -(p / D) * (G * a + phi(U) * b), rtol=1e-10, atol=1e-12)


# --- p = 2: textbook Laplacian closed forms ----------------------------------------------------

def pin_p2_closed_form(o):
    """At p = 2, F is the sum of Rayleigh quotients u^T L u / u^T u of the combinatorial
    Laplacian L = D - W (scipy), and the gradient and Hessian are the Rayleigh-quotient ones."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import laplacian

    rng = np.random.default_rng(15)
    n, k = 40, 3
    W = random_sym_weights(n, 0.15, rng)
    rp, c, w = csr_from_dense(W)
    Lap = laplacian(csr_matrix(W)).toarray()
    U = rng.standard_normal((n, k))
    V = rng.standard_normal((n, k))
    F, Fc, _, _ = o.objective(rp, c, w, U, 2.0)
    G, _ = o.grad(rp, c, w, U, 2.0)
    HV, G2, _ = o.hvp(rp, c, w, U, V, 2.0, 1e-8)
    for l in range(k):
        u, v = U[:, l], V[:, l]
        nu = u @ u
        R = u @ Lap @ u / nu
        assert abs(Fc[l] - R) <= 1e-12 * abs(R)
        g = 2.0 / nu * (Lap @ u - R * u)
        assert _rel(G[:, l], g) < 1e-12 and _rel(G2[:, l], g) < 1e-12
        Hv = 2.0 / nu * (Lap @ v - R * v - g * (u @ v) - u * (g @ v))
        assert _rel(HV[:, l], Hv) < 1e-12
    assert abs(F - sum(Fc)) < 1e-12 * abs(F)


# --- invariants of Eq. (1) ---------------------------------------------------------------------

def pin_invariants(o):
    """Scale/sign invariance of F, degree -1 homogeneity of G (hence H u = -g and <g, u> = 0),
    degree -2 homogeneity of H, symmetry of H, column separability, node relabelling, and the
    Euler identity sum_i u_i (Delta_p u)_i = N."""
    rng = np.random.default_rng(16)
    n, k = 30, 3
    W = random_sym_weights(n, 0.2, rng)
    rp, c, w = csr_from_dense(W)
    U = spread_block(n, k, rng)
    V = rng.standard_normal((n, k))
    X = rng.standard_normal((n, k))
    scale = np.array([2.5, -0.3, -1.7])
    perm_c = np.array([2, 0, 1])
    perm_n = rng.permutation(n)
    Wp = W[np.ix_(perm_n, perm_n)]
    rpp, cp, wp = csr_from_dense(Wp)
    eps = 1e-12
    for p in P_LEVELS:
        F, Fc, N, D = o.objective(rp, c, w, U, p)
        HV, G, _ = o.hvp(rp, c, w, U, V, p, eps)
        F2, _, _, _ = o.objective(rp, c, w, U * scale, p)
        assert abs(F2 - F) <= 1e-13 * abs(F)
        HV2, G2, _ = o.hvp(rp, c, w, U * scale, V, p, eps)
        assert _rel(G2 * scale, G) < 1e-12
        assert _rel(HV2 * scale ** 2, HV) < 1e-12
        assert np.max(np.abs(np.sum(G * U, axis=0))) <= 1e-12 * np.linalg.norm(G) * np.linalg.norm(U)
        HU, _, _ = o.hvp(rp, c, w, U, U, p, eps)
        assert _rel(HU, -G) < 1e-11
        HX, _, _ = o.hvp(rp, c, w, U, X, p, eps)
        for l in range(k):
            a, b = X[:, l] @ HV[:, l], V[:, l] @ HX[:, l]
            assert abs(a - b) <= 1e-11 * (abs(a) + abs(b) + 1e-300)
        HVc, Gc, Fcc = o.hvp(rp, c, w, U[:, perm_c], V[:, perm_c], p, eps)
        assert np.allclose(Fcc, Fc[perm_c], rtol=1e-14, atol=0) and _rel(Gc, G[:, perm_c]) < 1e-14
        assert _rel(HVc, HV[:, perm_c]) < 1e-14
        HVn, Gn, Fcn = o.hvp(rpp, cp, wp, U[perm_n], V[perm_n], p, eps)
        assert np.allclose(Fcn, Fc, rtol=1e-12, atol=0)
        assert _rel(Gn, G[perm_n]) < 1e-12 and _rel(HVn, HV[perm_n]) < 1e-12
        L = o.plap(rp, c, w, U, p)
        assert np.allclose(np.sum(U * L, axis=0), N, rtol=1e-12, atol=0)


def pin_disconnected(o):
    """Two components: per-component constant columns give F = 0 and G = 0 exactly; a constant
    column on a connected graph does too (every x = u_i - u_j is 0)."""
    rng = np.random.default_rng(17)
    W1 = random_sym_weights(6, 0.9, rng)
    W2 = random_sym_weights(5, 0.9, rng)
    W = np.zeros((11, 11))
    W[:6, :6] = W1
    W[6:, 6:] = W2
    rp, c, w = csr_from_dense(W)
    ind = np.zeros((11, 3))
    ind[:6, 0] = 1.0
    ind[6:, 1] = 1.0
    ind[:6, 2] = 2.0
    ind[6:, 2] = -0.5
    for p in P_LEVELS:
        F, Fc, _, _ = o.objective(rp, c, w, ind, p)
        assert F == 0.0 and np.all(Fc == 0.0)
        G, _ = o.grad(rp, c, w, ind, p)
        assert np.all(G == 0.0)
        rp1, c1, w1 = csr_from_dense(W1)
        F1, _, _, _ = o.objective(rp1, c1, w1, np.full((6, 1), 0.37), p)
        assert F1 == 0.0


def pin_eps_cap(o):
    """The regularised |x|^(p-2): with eps above every |u_i - u_j| and every |u_i|, each edge weight
    in the Hessian is w eps^(p-2), so H v equals the p = 2 Laplacian form scaled accordingly:
    (Hv)_i = (p/D)[(p-1) eps^(p-2) (L v)_i - F (p-1) eps^(p-2) v_i - g_i a - phi_p(u_i) b]."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import laplacian

    rng = np.random.default_rng(18)
    n = 12
    W = random_sym_weights(n, 0.5, rng)
    rp, c, w = csr_from_dense(W)
    Lap = laplacian(csr_matrix(W)).toarray()
    U = 1e-3 * spread_block(n, 1, rng)
    V = rng.standard_normal((n, 1))
    eps = 1.0
    for p in (1.6, 1.3, 1.1):
        HV, G, Fc = o.hvp(rp, c, w, U, V, p, eps)
        u, v, g = U[:, 0], V[:, 0], G[:, 0]
        D = np.sum(np.abs(u) ** p)
        phi = np.sign(u) * np.abs(u) ** (p - 1)
        cap = eps ** (p - 2)
        ref = (p / D) * ((p - 1) * cap * (Lap @ v) - Fc[0] * (p - 1) * cap * v - g * (phi @ v) - phi * (g @ v))
        assert _rel(HV[:, 0], ref) < 1e-12


# --- Grassmann steps -------------------------------------------------------------------------

def pin_projection(o=None):
    """P_U is the orthogonal projector onto the complement of span(U): U^T P_U(Z) = 0,
    P_U(P_U(Z)) = P_U(Z), P_U(U) = 0, and <P_U(Z), Y> = <Z, P_U(Y)>."""
    rng = np.random.default_rng(19)
    n, k = 50, 4
    U, _ = np.linalg.qr(rng.standard_normal((n, k)))
    Z = rng.standard_normal((n, k))
    Y = rng.standard_normal((n, k))
    P, M = orc.project(U, Z)
    assert np.max(np.abs(U.T @ P)) < 1e-13
    assert _rel(orc.project(U, P)[0], P) < 1e-13
    assert np.max(np.abs(orc.project(U, U)[0])) < 1e-13
    assert abs(np.sum(P * Y) - np.sum(Z * orc.project(U, Y)[0])) < 1e-12 * np.linalg.norm(Z) * np.linalg.norm(Y)
    assert np.max(np.abs(M - U.T @ Z)) < 1e-13


def _gram_schmidt(Y):
    """Classical Gram-Schmidt applied twice (independent of LAPACK's Householder QR)."""
    Q = np.array(Y, dtype=np.float64, copy=True)
    n, k = Q.shape
    for j in range(k):
        for _ in range(2):
            for i in range(j):
                Q[:, j] -= (Q[:, i] @ Q[:, j]) * Q[:, i]
        Q[:, j] /= np.linalg.norm(Q[:, j])
    return Q


def pin_retraction(o=None):
    """qf(U + t eta): orthonormal Q, R = Q^T Y upper triangular with positive diagonal, Q R = Y,
    equal to twice-applied Gram-Schmidt, and qf(U) = U for orthonormal U."""
    rng = np.random.default_rng(20)
    n, k = 60, 5
    U, _ = np.linalg.qr(rng.standard_normal((n, k)))
    eta, _ = orc.project(U, rng.standard_normal((n, k)))
    for t in (0.0, 0.1, 1.0, 7.5):
        Q = orc.retract(U, eta, t)
        Y = U + t * eta
        R = Q.T @ Y
        assert np.max(np.abs(Q.T @ Q - np.eye(k))) < 1e-13
        assert np.max(np.abs(np.tril(R, -1))) < 1e-12 * np.linalg.norm(Y)
        assert np.all(np.diag(R) > 0)
        assert _rel(Q @ R, Y) < 1e-13
        assert _rel(Q, _gram_schmidt(Y)) < 1e-11
    assert _rel(orc.retract(U, np.zeros_like(U), 1.0), U) < 1e-13


def pin_riemannian_hessian(o):
    """P_U(H eta) - eta (U^T G) equals the tangent part of the directional derivative of the
    gradient field X -> grad F(X) - X X^T grad F(X) along a tangent eta (central differences of
    the oracle gradient, itself pinned by pin_grad_fd)."""
    rng = np.random.default_rng(21)
    n, k = 25, 3
    W = random_sym_weights(n, 0.3, rng)
    rp, c, w = csr_from_dense(W)
    U, _ = np.linalg.qr(spread_block(n, k, rng))
    eta, _ = orc.project(U, rng.standard_normal((n, k)))
    h = 1e-6
    for p in (2.0, 1.5, 1.2):
        def field(X):
            Gx, _ = o.grad(rp, c, w, X, p)
            return Gx - X @ (X.T @ Gx)

        HV, G, _ = o.hvp(rp, c, w, U, eta, p, 1e-12)
        rh = orc.riemannian_hessian(U, G, HV, eta)
        fd, _ = orc.project(U, (field(U + h * eta) - field(U - h * eta)) / (2 * h))
        assert _rel(rh, fd) < 1e-6, (p, _rel(rh, fd))


ALL_PINS = [
    pin_two_node,
    pin_three_path,
    pin_brute_force,
    pin_grad_fd,
    pin_hvp_fd,
    pin_algorithm1_form,
    pin_p2_closed_form,
    pin_invariants,
    pin_disconnected,
    pin_eps_cap,
    pin_projection,
    pin_retraction,
    pin_riemannian_hessian,
    pin_hvp_sparse,
]


def failing_pins(o):
    """Names of the pins that the given oracle build fails (an exception counts as a failure)."""
    bad = []
    for pin in ALL_PINS:
        try:
            pin(o)
        except Exception:  # noqa: BLE001 - any failure of a mutant counts
            bad.append(pin.__name__)
    return bad
