"""Pins of the CPU oracle against what the paper and mathematics fix.

Each check below is independent of the oracle's own formulas: closed forms
derived from Eq. 2, symmetries (gauge covariance, H(mu)^dag = H(-mu)),
sign(A)^2 = I (the property stated after Eq. 6), the Hermitian mu = 0 case,
a library routine (scipy.linalg.signm) and brute force (Krylov on the full
space).  A plausible slip in the oracle (a dropped term, a wrong sign, a
misplaced U vs U^dag, a transposed operand) breaks at least one of them; the
mutation tests at the end plant such slips and check that they are caught.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import lattice_inputs as LI
import oracle as O
from oracle import dirac as OD


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ----------------------------------------------------------------- gamma basis
def test_gamma_algebra():
    g = O.gamma_matrices()
    for a in range(4):
        assert np.allclose(g[a], g[a].conj().T)
        for b in range(4):
            anti = g[a] @ g[b] + g[b] @ g[a]
            assert np.allclose(anti, 2.0 * np.eye(4) * (a == b))
    # gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 = diag(1,1,-1,-1) in the chiral basis
    assert np.allclose(g[4], np.diag([1, 1, -1, -1]))
    for a in range(4):
        assert np.allclose(g[4] @ g[a], -g[a] @ g[4])


def test_kappa():
    assert O.kappa_of(-1.5) == pytest.approx(0.2)
    assert O.kappa_of(-1.8) == pytest.approx(1.0 / 4.4)


# ------------------------------------------------------------ free-field pins
FREE_CASES = [((2, 2, 2, 2), 0.0, False), ((2, 2, 2, 2), 0.3, True),
              ((2, 2, 3, 4), 0.3, False), ((2, 3, 2, 4), 0.5, True),
              ((3, 3, 3, 3), 0.1, False)]


@pytest.mark.parametrize("dims,mu,ap", FREE_CASES)
def test_free_field_matvec(dims, mu, ap):
    """Explicit H_w(mu) on U = 1 equals the momentum-space H(p) of Eq. 2."""
    u = LI.make_links(dims, "unit")
    b = LI.gaussian_source(dims, cfg=0, inst=7)
    h = O.hermitian_wilson_sparse(u, dims, mu, -1.5, ap)
    assert rel(h @ b, O.free_field_h_apply(dims, mu, -1.5, b, ap)) < 1e-14


@pytest.mark.parametrize("dims,mu,ap", FREE_CASES[:4])
def test_free_field_sign_closed_form(dims, mu, ap):
    """Dense Newton sign(H) b equals H(p)/sqrt(s(p)) b on the free field."""
    u = LI.make_links(dims, "unit")
    b = LI.gaussian_source(dims, cfg=0, inst=8)
    h = O.hermitian_wilson_dense(u, dims, mu, -1.5, ap)
    y = O.sign_newton(h) @ b
    assert rel(y, O.free_field_sign_apply(dims, mu, -1.5, b, ap)) < 1e-12


def test_free_field_spectrum():
    dims, mu = (2, 2, 3, 4), 0.3
    h = O.hermitian_wilson_dense(LI.make_links(dims, "unit"), dims, mu, -1.5)
    ev = np.linalg.eigvals(h)
    ref = O.free_field_spectrum(dims, mu, -1.5)
    # every eigenvalue has a closed-form partner (multiset match by greedy pairing)
    ref = list(ref)
    for e in ev:
        j = int(np.argmin(np.abs(np.asarray(ref) - e)))
        assert abs(ref[j] - e) < 1e-9
        ref.pop(j)


# ------------------------------------------------------------------ symmetries
def _haar_case(dims=(2, 2, 2, 2), inst=0):
    return LI.make_links(dims, "haar", cfg=0, inst=inst)


def test_adjoint_identity():
    """H_w(mu)^dag = H_w(-mu): gamma_5 Hermitian, backward hops carry U^dag e^{-mu}."""
    dims = (2, 3, 2, 3)
    u = _haar_case(dims)
    hp = O.hermitian_wilson_sparse(u, dims, 0.4, -1.5)
    hm = O.hermitian_wilson_sparse(u, dims, -0.4, -1.5)
    assert abs(hp.conj().T - hm).max() < 1e-15


def test_gauge_covariance():
    """U_{n,nu} -> g_n U_{n,nu} g_{n+nu}^dag gives H -> G H G^dag."""
    dims = (2, 3, 2, 3)
    u = _haar_case(dims, inst=3)
    g = LI.haar_su3(LI.rng_for(0, 99, 0), LI.volume(dims))
    up = np.empty_like(u)
    for nu in range(4):
        fwd, _ = OD.neighbour(dims, nu, +1)
        up[:, nu] = g @ u[:, nu] @ np.conj(np.transpose(g[fwd], (0, 2, 1)))
    gm = np.zeros((12 * len(g), 12 * len(g)), dtype=complex)
    for n in range(len(g)):
        gm[12 * n:12 * n + 12, 12 * n:12 * n + 12] = np.kron(np.eye(4), g[n])
    h = O.hermitian_wilson_dense(u, dims, 0.3, -1.5)
    hp = O.hermitian_wilson_dense(up, dims, 0.3, -1.5)
    assert np.abs(hp - gm @ h @ gm.conj().T).max() < 1e-13


def test_mu_zero_hermitian_and_unitary_sign():
    dims = (2, 2, 2, 2)
    h = O.hermitian_wilson_dense(_haar_case(dims), dims, 0.0, -1.5)
    assert np.abs(h - h.conj().T).max() < 1e-15
    w, vec = np.linalg.eigh(h)
    s_ref = vec @ np.diag(np.sign(w)) @ vec.conj().T
    s = O.sign_newton(h)
    assert np.abs(s - s_ref).max() < 1e-12
    assert np.abs(s - s.conj().T).max() < 1e-12
    assert np.abs(s @ s.conj().T - np.eye(len(h))).max() < 1e-12


# -------------------------------------------------------------- dense routes
@pytest.fixture(scope="module")
def haar2():
    dims = (2, 2, 2, 2)
    u = _haar_case(dims, inst=1)
    h = O.hermitian_wilson_dense(u, dims, 0.3, -1.5)
    return dims, u, h


def test_sign_routes_agree(haar2):
    _, _, h = haar2
    sn, info = O.sign_newton(h, return_info=True)
    se, einfo = O.sign_eig(h, return_info=True)
    assert rel(sn, se) < 1e-11
    assert rel(sn, sla.signm(h)) < 1e-9        # library routine, looser by design
    assert info["x2_minus_i"] < 1e-12          # sign(A)^2 = I
    assert einfo["min_abs_re"] > 1e-3


def test_sign_commutes_with_h(haar2):
    dims, _, h = haar2
    b = LI.gaussian_source(dims, cfg=0, inst=2)
    s = O.sign_newton(h)
    assert rel(s @ (h @ b), h @ (s @ b)) < 1e-12


def test_adjoint_sign_identity(haar2):
    """<a, S(mu) b> = <S(-mu) a, b> from H(mu)^dag = H(-mu)."""
    dims, u, h = haar2
    hm = O.hermitian_wilson_dense(u, dims, -0.3, -1.5)
    a = LI.gaussian_source(dims, cfg=0, inst=3)
    b = LI.gaussian_source(dims, cfg=0, inst=4)
    lhs = np.vdot(a, O.sign_newton(h) @ b)
    rhs = np.vdot(O.sign_newton(hm) @ a, b)
    assert abs(lhs - rhs) < 1e-12


def test_sgn_scalar():
    z = np.array([1 + 5j, -1e-3 + 2j, 2.0, -3.0 - 1j])
    assert np.allclose(O.sgn(z), [1, -1, 1, -1])
    # sgn(z) = z / sqrt(z^2) with the principal square root (Eq. 5)
    assert np.allclose(z / np.sqrt(z * z), O.sgn(z))


# ---------------------------------------------------------------- Krylov pins
def test_arnoldi_relation(haar2):
    dims, _, h = haar2
    b = LI.gaussian_source(dims, cfg=0, inst=5)
    k = 40
    vmat, hmat, beta, kd = O.arnoldi_cgs2(lambda x: h @ x, b, k)
    assert kd == k
    assert np.abs(vmat.conj().T @ vmat - np.eye(k + 1)).max() < 1e-13
    assert np.abs(h @ vmat[:, :k] - vmat @ hmat).max() < 1e-13
    assert np.allclose(np.tril(hmat, -2), 0)
    assert np.all(np.abs(np.diag(hmat, -1).imag) == 0) and np.all(np.diag(hmat, -1).real > 0)


def test_krylov_full_space_is_exact(haar2):
    """Krylov with k = N (or a happy breakdown) reproduces the dense sign."""
    dims, _, h = haar2
    b = LI.gaussian_source(dims, cfg=0, inst=6)
    y, info = O.lr_arnoldi_sign(lambda x: h @ x, b, None, k=h.shape[0], route="eig")
    assert rel(y, O.sign_newton(h) @ b) < 1e-10


def test_krylov_breakdown_on_free_plane_wave():
    """A free-field plane wave spans a tiny invariant space: happy breakdown, exact."""
    dims = (2, 2, 2, 4)
    u = LI.make_links(dims, "unit")
    h = O.hermitian_wilson_dense(u, dims, 0.3, -1.5)
    lx, ly, lz, lt = dims
    t = np.arange(lt)
    wave = np.exp(2j * np.pi * t / lt)[:, None, None, None, None, None] * np.ones((1, lz, ly, lx, 4, 3))
    chi = np.zeros((4, 3), dtype=complex)
    chi[0, 0] = 1.0
    b = (wave * chi).reshape(-1)
    b /= np.linalg.norm(b)
    y, info = O.lr_arnoldi_sign(lambda x: h @ x, b, None, k=50)
    assert info["k_used"] <= 4
    assert rel(y, O.sign_newton(h) @ b) < 1e-12


def test_small_sign_routes_agree(haar2):
    dims, _, h = haar2
    b = LI.gaussian_source(dims, cfg=0, inst=9)
    _, hmat, _, _ = O.arnoldi_cgs2(lambda x: h @ x, b, 60)
    hk = hmat[:60, :60]
    assert rel(O.small_sign_e1(hk, "newton"), O.small_sign_e1(hk, "eig")) < 1e-10


# ------------------------------------------------------------ LR deflation
@pytest.fixture(scope="module")
def haar3():
    dims = (3, 3, 3, 3)
    u = LI.make_links(dims, "haar", cfg=0, inst=11)
    h = O.hermitian_wilson_dense(u, dims, 0.3, -1.5)
    b = LI.gaussian_source(dims, cfg=0, inst=11)
    y = O.sign_eig_apply(h, b)
    return dims, u, h, b, y


def test_lr_projector_properties(haar3):
    dims, u, h, b, y = haar3
    r, l, lam = O.critical_dense(h, 12)
    defl = O.Deflation(r, l, lam)
    assert np.abs(defl.g - np.eye(12)).max() < 1e-10           # L^dag R = I (Eq. 20 text)
    assert np.abs(h @ r - r * lam).max() < 1e-12               # A R = R Lambda
    assert np.abs(l.conj().T @ h - lam[:, None] * l.conj().T).max() < 1e-11
    c, xo = defl.split(b)
    assert np.abs(l.conj().T @ xo).max() < 1e-12               # x_ominus has no critical part
    # Eq. 21 holds exactly: f(A) b = R f(Lambda) L^dag b + f(A) x_ominus
    assert rel(defl.exact_part(c) + O.sign_eig_apply(h, xo), y) < 1e-11
    # critical eigenvalues have the smallest |Re|
    allev = np.linalg.eigvals(h)
    assert np.max(np.abs(lam.real)) <= np.sort(np.abs(allev.real))[12] + 1e-12


def test_lr_deflation_accelerates(haar3):
    """Error falls with k, and deflation lowers it at fixed k (Results section trends)."""
    dims, u, h, b, y = haar3
    mv = lambda x: h @ x  # noqa: E731
    errs = {}
    for m in (0, 8, 24):
        defl = O.Deflation(*O.critical_dense(h, m)) if m else None
        errs[m] = [rel(O.lr_arnoldi_sign(mv, b, defl, k=k)[0], y) for k in (40, 80, 160)]
    for m in errs:
        assert errs[m][0] > errs[m][1] > errs[m][2]
    assert errs[24][1] < errs[8][1] < errs[0][1]
    assert errs[24][2] < 1e-7


def test_lr_near_best_approximation(haar3):
    """The LR result is close to the orthogonal projection of f(A)b on Omega_m + K_k."""
    dims, u, h, b, y = haar3
    r, l, lam = O.critical_dense(h, 12)
    defl = O.Deflation(r, l, lam)
    k = 60
    yk, info = O.lr_arnoldi_sign(lambda x: h @ x, b, defl, k=k)
    _, xo = defl.split(b)
    vmat, _, _, _ = O.arnoldi_cgs2(lambda x: h @ x, xo, k)
    q, _ = np.linalg.qr(np.concatenate([r, vmat[:, :k]], axis=1))
    best = q @ (q.conj().T @ y)
    assert np.linalg.norm(yk - y) < 20 * np.linalg.norm(best - y)


def test_hermitian_deflation_special_case():
    """At mu = 0 LR deflation reduces to Eq. 12: L = R orthonormal, G = I."""
    dims = (2, 2, 3, 3)
    u = LI.make_links(dims, "haar", cfg=0, inst=12)
    h = O.hermitian_wilson_dense(u, dims, 0.0, -1.5)
    r, l, lam = O.critical_dense(h, 10)
    assert np.abs(lam.imag).max() < 1e-12
    assert np.abs(r.conj().T @ r - np.eye(10)).max() < 1e-10
    assert np.abs(l - r).max() < 1e-10


def test_critical_sparse_matches_dense(haar3):
    dims, u, h, b, y = haar3
    hs = O.hermitian_wilson_sparse(u, dims, 0.3, -1.5)
    hm = O.hermitian_wilson_sparse(u, dims, -0.3, -1.5)
    r1, l1, lam1 = O.critical_dense(h, 10)
    r2, l2, lam2 = O.critical_sparse(hs, hm, 10)
    assert np.abs(np.sort_complex(lam1) - np.sort_complex(lam2)).max() < 1e-10
    # the oblique projector R G^{-1} L^dag is canonical
    p1 = O.Deflation(r1, l1, lam1)
    p2 = O.Deflation(r2, l2, lam2)
    assert rel(p2.r @ p2.coeffs(b), p1.r @ p1.coeffs(b)) < 1e-9
    assert max(O.eig_residuals(h, r2, l2, lam2)) < 1e-10


def test_monitor_stops_early(haar3):
    dims, u, h, b, y = haar3
    defl = O.Deflation(*O.critical_dense(h, 24))
    yk, info = O.lr_arnoldi_sign(lambda x: h @ x, b, defl, k=400, check=10, tol=1e-9)
    assert info["k_used"] < 400 and info["est"] <= 1e-9
    assert rel(yk, y) < 1e-7


# ------------------------------------------------- planted mistakes are caught
def test_planted_mu_sign_flip_is_caught(monkeypatch):
    """Swapping e^{+mu} and e^{-mu} in the oracle breaks the free-field pin."""
    dims, mu = (2, 2, 2, 4), 0.3
    u = LI.make_links(dims, "unit")
    b = LI.gaussian_source(dims, cfg=0, inst=13)
    wrong = O.hermitian_wilson_sparse(u, dims, -mu, -1.5)
    assert rel(wrong @ b, O.free_field_h_apply(dims, mu, -1.5, b)) > 1e-3


def test_planted_link_adjoint_slip_is_caught(monkeypatch):
    """Using U instead of U^dag on the backward hop breaks H(mu)^dag = H(-mu)
    and gauge covariance."""
    dims = (2, 3, 2, 3)
    u = _haar_case(dims, inst=3)
    monkeypatch.setattr(OD, "_backward_link", lambda links, bwd, nu: links[bwd, nu])
    hp = O.hermitian_wilson_sparse(u, dims, 0.4, -1.5)
    hm = O.hermitian_wilson_sparse(u, dims, -0.4, -1.5)
    assert abs(hp.conj().T - hm).max() > 1e-3


def test_planted_dropped_diagonal_is_caught(monkeypatch):
    """Dropping the e^{-mu} factor (a plausible slip) breaks the free-field pin."""
    dims, mu = (2, 2, 2, 4), 0.3
    u = LI.make_links(dims, "unit")
    b = LI.gaussian_source(dims, cfg=0, inst=14)
    real_exp = np.exp
    monkeypatch.setattr(OD.np, "exp", lambda x: 1.0 if np.isscalar(x) and x < 0 else real_exp(x))
    h = O.hermitian_wilson_sparse(u, dims, mu, -1.5)
    monkeypatch.undo()
    assert rel(h @ b, O.free_field_h_apply(dims, mu, -1.5, b)) > 1e-3


# ------------------------------------------------- overlap operator and adjoint
def _tiny(mu):
    dims = (2, 2, 2, 2)
    links = LI.make_links(dims, "haar", cfg=7, inst=3)
    return dims, links, O.hermitian_wilson_dense(links, dims, mu, -1.5)


def _as_matrix(apply, n):
    return apply(np.eye(n, dtype=complex))


def test_adjoint_sign_is_the_adjoint():
    """<a, sign(H) b> = <sign(H)^dag a, b>, sign(H)^dag from an eigendecomposition of
    H^dag independent of the one of H; and H(mu)^dag = H(-mu) gives the same vector."""
    dims, links, h = _tiny(0.4)
    rng = np.random.default_rng(11)
    n = h.shape[0]
    a = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    lhs = np.vdot(a, O.sign_eig_apply(h, b))
    rhs = np.vdot(O.sign_adjoint_apply(h, a), b)
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)
    h_minus = O.hermitian_wilson_dense(links, dims, -0.4, -1.5)
    assert rel(O.sign_adjoint_apply(h, a), O.sign_eig_apply(h_minus, a)) < 1e-11


def test_overlap_ginsparg_wilson_circle_and_gamma5_hermiticity():
    """At mu = 0 sign(H) is Hermitian and unitary, so the spectrum of D_ov lies on
    |z - 1| = 1; at any mu, D_ov(mu)^dag = gamma_5 D_ov(-mu) gamma_5."""
    dims, links, h0 = _tiny(0.0)
    n = h0.shape[0]
    d0 = _as_matrix(lambda x: O.overlap_apply(h0, x), n)
    ev = np.linalg.eigvals(d0)
    assert np.max(np.abs(np.abs(ev - 1.0) - 1.0)) < 1e-10
    _, _, hp = _tiny(0.3)
    _, _, hm = _tiny(-0.3)
    dp = _as_matrix(lambda x: O.overlap_apply(hp, x), n)
    dm = _as_matrix(lambda x: O.overlap_apply(hm, x), n)
    g5 = np.diag(OD.gamma5_diag(n // 12))
    assert np.abs(dp.conj().T - g5 @ dm @ g5).max() < 1e-10
    # (gamma_5 (D_ov - 1))^2 = sign(H)^2 = 1 (the property after Eq. 6)
    q = g5 @ (dp - np.eye(n))
    assert np.abs(q @ q - np.eye(n)).max() < 1e-9


# ------------------------------------------------------------ Schur deflation
def test_schur_basis_relation(haar3):
    """Eq. 13: S_m orthonormal, A S_m = S_m T_m, T_m upper triangular with the
    critical eigenvalues on its diagonal; it agrees with scipy's sorted complex
    Schur form up to a unitary diagonal (its eigenvalues are distinct)."""
    dims, u, h, b, y = haar3
    r, l, lam = O.critical_dense(h, 10)
    s, t = O.schur_basis(r, lambda x: h @ x)
    assert np.abs(s.conj().T @ s - np.eye(10)).max() < 1e-12
    assert np.abs(h @ s - s @ t).max() < 1e-11
    assert np.abs(np.tril(t, -1)).max() < 1e-11
    assert np.abs(np.diag(t) - lam).max() < 1e-11
    # the same invariant subspace from an independent Schur factorisation of A
    thr = np.max(np.abs(lam.real))
    ts, zs, sdim = sla.schur(h, output="complex", sort=lambda z: abs(z.real) <= thr + 1e-13)
    assert sdim == 10
    zs = zs[:, :10]
    assert np.abs(zs @ (zs.conj().T @ s) - s).max() < 1e-10


def test_schur_full_space_is_exact(haar2):
    """With the Krylov space filling the orthogonal complement (k = N - m) the
    Eq. 19 approximation is sign(A) b to rounding, for several m."""
    dims, u, h = haar2
    rng = np.random.default_rng(5)
    n = h.shape[0]
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    yx = O.sign_eig_apply(h, b)
    for m in (0, 4, 12):
        r = O.critical_dense(h, m)[0] if m else np.zeros((n, 0), complex)
        s, t = O.schur_basis(r, lambda x: h @ x)
        y, info = O.schur_arnoldi_sign(lambda x: h @ x, b, s, t, k=n - m)
        assert rel(y, yx) < 1e-9, m


def test_schur_block_sign_and_sylvester(haar3):
    """Eq. 17-18: the sign of the block matrix H = [[T, X], [0, H_k]], taken whole
    by its eigendecomposition, has f(T), Y and f(H_k) as its blocks."""
    dims, u, h, b, y = haar3
    r = O.critical_dense(h, 8)[0]
    s, t = O.schur_basis(r, lambda x: h @ x)
    yk, info = O.schur_arnoldi_sign(lambda x: h @ x, b, s, t, k=40)
    k = info["k_used"]
    big = np.block([[t, info["x"]], [np.zeros((k, 8)), info["hk"][:k, :k]]])
    fb = O.sign_eig(big)
    assert np.abs(fb[:8, :8] - info["fT"]).max() < 1e-9
    assert np.abs(fb[8:, 8:] - info["fH"]).max() < 1e-9
    assert np.abs(fb[:8, 8:] - info["y_coupling"]).max() < 1e-9
    assert np.abs(fb[8:, :8]).max() < 1e-12
    # the Arnoldi relation of Eq. 14 with the composite basis
    vmat, hm, xm, beta, c0, kd = O.schur_arnoldi(lambda x: h @ x, b, s, 40)
    q = np.concatenate([s, vmat[:, :kd]], axis=1)
    hq = np.block([[t, xm], [np.zeros((kd, 8)), hm[:kd, :kd]]])
    resid = h @ q - q @ hq
    resid[:, -1] -= hm[kd, kd - 1] * vmat[:, kd]
    assert np.abs(resid).max() < 1e-11
    assert np.abs(q.conj().T @ q - np.eye(8 + kd)).max() < 1e-12


def test_schur_basis_invariance_and_special_cases(haar3):
    """Eq. 19 depends on Omega_m, not on the basis: S -> S W, T -> W^dag T W with W
    unitary (T no longer triangular) gives the same vector.  m = 0 reduces to the
    plain Arnoldi approximation; a source inside Omega_m is mapped exactly."""
    dims, u, h, b, y = haar3
    mv = lambda x: h @ x  # noqa: E731
    r, l, lam = O.critical_dense(h, 8)
    s, t = O.schur_basis(r, mv)
    y1, _ = O.schur_arnoldi_sign(mv, b, s, t, k=50)
    w, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((8, 8))
                        + 1j * np.random.default_rng(4).standard_normal((8, 8)))
    y2, _ = O.schur_arnoldi_sign(mv, b, s @ w, w.conj().T @ t @ w, k=50)
    assert rel(y2, y1) < 1e-10
    n = h.shape[0]
    y0, _ = O.schur_arnoldi_sign(mv, b, np.zeros((n, 0), complex), np.zeros((0, 0)), k=50)
    assert rel(y0, O.lr_arnoldi_sign(mv, b, None, k=50)[0]) < 1e-11
    xin = r @ np.arange(1, 9)
    yin, info = O.schur_arnoldi_sign(mv, xin, s, t, k=10)
    assert info["k_used"] == 0 and rel(yin, O.sign_eig_apply(h, xin)) < 1e-10


def test_schur_accuracy_close_to_lr(haar3):
    """Results section: Schur deflation is about as accurate as LR deflation at
    equal (m, k); both improve on no deflation."""
    dims, u, h, b, y = haar3
    mv = lambda x: h @ x  # noqa: E731
    r, l, lam = O.critical_dense(h, 16)
    s, t = O.schur_basis(r, mv)
    for k in (60, 120):
        es = rel(O.schur_arnoldi_sign(mv, b, s, t, k=k)[0], y)
        el = rel(O.lr_arnoldi_sign(mv, b, O.Deflation(r, l, lam), k=k)[0], y)
        e0 = rel(O.lr_arnoldi_sign(mv, b, None, k=k)[0], y)
        assert es < e0 and el < e0
        assert 0.1 < es / el < 10.0, (k, es, el)


# ------------------------------------------------------------ block Krylov
def test_block_arnoldi_relation_and_single_source(haar2):
    """Block Arnoldi: A V_K = V_K H_K + V_{K+1} H_{K+1,K} E_K^T with orthonormal V and
    block upper Hessenberg H; with one source the block method is Eq. 22."""
    dims, u, h = haar2
    n = h.shape[0]
    rng = np.random.default_rng(8)
    b = rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))
    mvb = lambda x: h @ x  # noqa: E731
    vmat, hmat, r0, kd = O.block_arnoldi(mvb, b, 12)
    s = 3
    assert kd == 12
    assert np.abs(vmat.conj().T @ vmat - np.eye((kd + 1) * s)).max() < 1e-12
    resid = h @ vmat[:, : kd * s] - vmat @ hmat
    assert np.abs(resid).max() < 1e-11
    assert np.abs(np.tril(hmat, -s - 1)).max() == 0.0            # block Hessenberg
    assert np.abs(vmat[:, :s] @ r0 - b).max() < 1e-12
    r, l, lam = O.critical_dense(h, 6)
    defl = O.Deflation(r, l, lam)
    y1, _ = O.block_lr_sign(lambda x: h @ x, b[:, :1], defl, 30)
    y2, _ = O.lr_arnoldi_sign(lambda x: h @ x, b[:, 0], defl, k=30)
    assert rel(y1[:, 0], y2) < 1e-10


def test_block_krylov_exact_on_full_space_and_contains_single_spaces(haar2):
    """When K s reaches the complement's dimension the block result is the exact
    sign; the block space of K steps contains each source's own Krylov space of K
    steps, so its error at K is no worse than the single-source error at K."""
    dims, u, h = haar2
    n = h.shape[0]
    rng = np.random.default_rng(9)
    b = rng.standard_normal((n, 4)) + 1j * rng.standard_normal((n, 4))
    yx = O.sign_eig_apply(h, b)
    r, l, lam = O.critical_dense(h, 8)
    defl = O.Deflation(r, l, lam)
    yb, info = O.block_lr_sign(lambda x: h @ x, b, defl, (n - 8) // 4)
    assert rel(yb, yx) < 1e-9
    for k in (6, 12):
        yb, _ = O.block_lr_sign(lambda x: h @ x, b, defl, k)
        for i in range(4):
            ys, _ = O.lr_arnoldi_sign(lambda x: h @ x, b[:, i], defl, k=k)
            assert rel(yb[:, i], yx[:, i]) < 3 * rel(ys, yx[:, i]), (k, i)


def test_newton_schulz_tail_reading(haar2):
    """The small-sign reading used on the GPU: once |X^2 - I|_F < 0.5, Newton-Schulz
    steps X <- (3X - X^3)/2 from a Newton iterate converge to the same sign as the
    spectral definition; without that condition an eigenvalue beyond sqrt(3) is
    flipped (2 -> -1), which is why the check is needed."""
    dims, u, h = haar2
    x = np.array(h, dtype=complex)
    eye = np.eye(len(h))
    for _ in range(60):                       # plain Newton until the condition holds
        if np.linalg.norm(x @ x - eye) < 0.5:
            break
        x = 0.5 * (x + np.linalg.inv(x))
    assert np.linalg.norm(x @ x - eye) < 0.5
    for _ in range(30):
        x = 0.5 * (3 * x - x @ x @ x)
    assert np.abs(x - O.sign_eig(h)).max() < 1e-10
    assert 0.5 * (3 * 2.0 - 2.0 ** 3) == -1.0


def _geometric_rate(e1, d1, e2, d2):
    """The rate the GPU's stopping rule solves for: e2 / e1 = r^d1 (1 - r^d2) / (1 - r^d1)."""
    if not (e1 > 0) or e2 < 0:
        return 1.0
    if e2 == 0:
        return 0.0
    ratio = e2 / e1
    if not ratio < 0.999 * d2 / d1:
        return 1.0
    lo, hi = 0.0, 1.0
    for _ in range(80):
        r = 0.5 * (lo + hi)
        f = r ** d1 * (1 - r ** d2) / (1 - r ** d1)
        lo, hi = (r, hi) if f < ratio else (lo, r)
    return hi


@pytest.mark.parametrize("kind,eps", [("haar", 0.0), ("disordered", 0.9)])
def test_geometric_tail_estimate_reading(kind, eps):
    """The GPU's default convergence estimate (the paper gives no stopping rule):
    at checks every d Arnoldi steps the change c_k = beta |s_k - [s_{k-d}; 0]| / |b|
    of the Krylov iterate (Eq. 22) is about the error of check k - d.  Two
    successive changes give the per-step rate r of a geometric error, and twice
    the tail c_k r^d / (1 - r^d), with the slower of the last two rates, is the
    estimate of the error of check k.  On the oracle's own iterates it must not
    fall below the true error (against the spectral sign, Eq. 4-6) once the
    error is in the asymptotic regime (below 1e-4, where stopping decisions for
    practical tolerances are taken; far from convergence the error can stall
    for a check while the change is large) and above rounding, and the first
    check where it is <= 1e-8 must have a true error <= 1e-8."""
    dims = (2, 3, 3, 4)
    links = LI.make_links(dims, kind, eps=eps, cfg=9, inst=40)
    b = LI.gaussian_source(dims, cfg=9, inst=40)
    h = O.hermitian_wilson_dense(links, dims, 0.3, -1.5)
    yex = O.sign_eig_apply(h, b)
    defl = O.Deflation(*O.critical_dense(h, 6))
    c, xo = defl.split(b)
    vmat, hmat, beta, kd = O.arnoldi_cgs2(lambda x: h @ x, xo, 500, project=defl.project_out)
    bn = np.linalg.norm(b)
    ys, ss = {}, {}
    for d in (10, 25):
        prev_s, changes, rates, stop_err = None, [], [], None
        for k in range(d, kd + 1, d):
            if k not in ss:
                ss[k] = O.small_sign_e1(hmat[:k, :k], "eig")
                ys[k] = defl.exact_part(c) + beta * (vmat[:, :k] @ ss[k])
            s, y = ss[k], ys[k]
            err = rel(y, yex)
            if prev_s is not None:
                ds = s.copy()
                ds[: prev_s.size] -= prev_s
                ch = beta * np.linalg.norm(ds) / bn
                tail = ch
                if changes:
                    r = _geometric_rate(changes[-1], d, ch, d)
                    r_use = max([r] + rates[-1:])
                    rates.append(r)
                    q = r_use ** d
                    tail = 2 * ch * q / (1 - q) if q < 1 else np.inf
                changes.append(ch)
                est = tail * bn / np.linalg.norm(y)
                if 1e-12 < err < 1e-4 and len(changes) >= 2:
                    assert est >= err, (d, k, est, err)
                if stop_err is None and est <= 1e-8:
                    stop_err = err
            prev_s = s
        assert stop_err is not None and stop_err <= 1e-8, d


def _two_step_arnoldi(matvec, x, k, project=None, merged=False):
    """The GPU's two-step block form of the Arnoldi recurrence, written out in
    numpy: per outer step W = [H u_b, H^2 u_b] from the last unfinished vector;
    one set of inner products [V, U]^H [U, W]; U finished by its second
    Gram-Schmidt pass and a 2x2 Cholesky factor R; W orthogonalised once; the
    Hessenberg columns recovered from R and the first-pass coefficients.
    merged: the re-projection of both columns of W after H^2 u_b = H (H u_b)
    (the GPU's order), instead of projecting after each application."""
    prj0 = project if project else (lambda v: v)

    def block(v):
        if merged:
            w1 = matvec(v)
            return np.stack([prj0(w1), prj0(matvec(w1))], 1)
        w1 = prj0(matvec(v))
        return np.stack([w1, prj0(matvec(w1))], 1)

    n_all = x.shape[0]
    beta = np.linalg.norm(x)
    vmat = np.zeros((n_all, k + 3), dtype=complex)
    hmat = np.zeros((k + 3, k + 2), dtype=complex)
    vmat[:, 0] = x / beta
    w = block(vmat[:, 0])
    cv = vmat[:, :1].conj().T @ w
    u = w - vmat[:, :1] @ cv
    n, a, t0, cp = 1, cv[:, 0].copy(), 1.0, cv.copy()
    while n + 1 <= k:
        w = block(u[:, 1])
        vn = vmat[:, :n]
        s, g = vn.conj().T @ u, u.conj().T @ u
        cvn, e = vn.conj().T @ w, u.conj().T @ w
        r = np.linalg.cholesky(g - s.conj().T @ s).conj().T
        q = (u - vn @ s) @ np.linalg.inv(r)
        vmat[:, n:n + 2] = q
        cq = np.linalg.solve(r.conj().T, e - s.conj().T @ cvn)
        u_next = w - vn @ cvn - q @ cq
        hmat[:n, n - 1] = a + t0 * s[:, 0]
        hmat[n, n - 1] = t0 * r[0, 0]
        col = np.zeros(n + 2, dtype=complex)
        col[:n] = cp[:, 1] + s[:, 1]
        col[n], col[n + 1] = r[0, 1], r[1, 1]
        col[:n + 1] -= hmat[:n + 1, :n] @ (cp[:, 0] + s[:, 0])
        hmat[:n + 2, n] = col / r[0, 0]
        a = np.concatenate([cvn[:, 0], cq[:, 0]])
        a[:n + 1] -= hmat[:n + 1, :n] @ s[:, 1]
        a -= hmat[:n + 2, n] * r[0, 1]
        a /= r[1, 1]
        t0, cp, u = 1.0 / r[1, 1].real, np.vstack([cvn, cq]), u_next
        n += 2
    kk = n - 1
    return vmat[:, :kk + 1], hmat[:kk + 1, :kk], beta, kk


@pytest.mark.parametrize("kind,mu,m,merged", [("haar", 0.3, 0, False),
                                              ("disordered", 0.5, 8, False),
                                              ("disordered", 0.5, 8, True)])
def test_two_step_arnoldi_reading(kind, mu, m, merged):
    """The two-step block form (the GPU's orth 2) builds the Arnoldi
    decomposition of Eq. 7 that the oracle's CGS2 recurrence builds: the
    decomposition with v_1 = x/|x| and a real positive subdiagonal is unique,
    so the Hessenberg matrices, the bases and Eq. 22 agree to rounding, with
    and without LR deflation and the per-vector re-projection, also with both
    new columns projected together after the second application of H (H
    commutes with the LR projector, Eq. 21)."""
    dims = (3, 4, 3, 4)
    links = LI.make_links(dims, kind, eps=0.6, cfg=9, inst=41)
    b = LI.gaussian_source(dims, cfg=9, inst=41)
    h = O.hermitian_wilson_sparse(links, dims, mu, -1.5)
    defl = O.Deflation(*O.critical_dense(h.toarray(), m)) if m else None
    xo = defl.split(b)[1] if defl else b
    proj = defl.project_out if defl else None
    k = 120
    v2, h2, b2, k2 = _two_step_arnoldi(lambda v: h @ v, xo, k, proj, merged)
    vo, ho, bo, ko = O.arnoldi_cgs2(lambda v: h @ v, xo, k, project=proj)
    assert k2 == ko == k
    assert np.abs(v2.conj().T @ v2 - np.eye(k + 1)).max() < 1e-13
    assert np.abs(h2 - ho).max() < 1e-12 * np.abs(ho).max()
    assert np.abs(v2 - vo).max() < 1e-11
    y2 = b2 * v2[:, :k] @ O.small_sign_e1(h2[:k, :k])
    yo = bo * vo[:, :k] @ O.small_sign_e1(ho[:k, :k])
    assert rel(y2, yo) < 1e-12
