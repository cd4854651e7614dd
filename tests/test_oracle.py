"""Pins of the FP64 oracle against what the mathematics fixes independently of it.

Each test checks an oracle function against a closed form, an invariant, a
brute-force evaluation on a tiny grid or a finite difference, chosen so that a
dropped term, a wrong sign or index, or a transposed operand fails one of them.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_0904_4887_amd import workloads as W

FOUR_PI = 4.0 * math.pi


def _rand_case(shape, seed, eps_hi=78.36):
    rng = np.random.default_rng(seed)
    eps = rng.uniform(1.0, eps_hi, size=shape)
    rho = rng.normal(size=shape)
    rho -= rho.mean()
    return eps, rho


# ---------------------------------------------------------------- operator A

def _bilinear_by_faces(phi, psi, eps, h):
    """-sum over every face f of eps_f (D_f phi)(D_f psi): the quadratic form
    whose Hessian defines the conservative operator (pure-Python loops)."""
    nz, ny, nx = phi.shape
    tot = 0.0
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                for di, dj, dk, hd in ((1, 0, 0, h[0]), (0, 1, 0, h[1]), (0, 0, 1, h[2])):
                    k2, j2, i2 = (k + dk) % nz, (j + dj) % ny, (i + di) % nx
                    ef = 0.5 * (eps[k, j, i] + eps[k2, j2, i2])
                    tot += ef * (phi[k2, j2, i2] - phi[k, j, i]) * (psi[k2, j2, i2] - psi[k, j, i]) / hd ** 2
    return -tot


def test_apply_A_matches_face_bilinear_form():
    h = (0.3, 0.45, 0.7)
    rng = np.random.default_rng(3)
    shape = (3, 4, 5)
    eps = rng.uniform(1.0, 78.0, size=shape)
    for _ in range(3):
        phi, psi = rng.normal(size=shape), rng.normal(size=shape)
        lhs = float(np.sum(psi * O.apply_A(phi, eps, h)))
        rhs = _bilinear_by_faces(phi, psi, eps, h)
        assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


def test_apply_A_null_space_and_symmetry():
    h = (0.2, 0.25, 0.3)
    eps, _ = _rand_case((6, 5, 7), 1)
    assert np.abs(O.apply_A(np.ones_like(eps), eps, h)).max() < 1e-10
    rng = np.random.default_rng(2)
    u, v = rng.normal(size=eps.shape), rng.normal(size=eps.shape)
    a = np.sum(u * O.apply_A(v, eps, h))
    b = np.sum(v * O.apply_A(u, eps, h))
    assert abs(a - b) <= 1e-12 * abs(a)
    assert np.sum(u * O.apply_A(u, eps, h)) < 0.0


def test_single_fourier_mode_eigenvalue():
    """A cosine mode is an eigenvector of the uniform-eps 7-point operator with
    eigenvalue -eps sum_d (2 - 2 cos(2 pi m_d / n_d)) / h_d^2 = -eps sum_d 4 sin^2(pi m_d/n_d)/h_d^2."""
    n = (12, 10, 8)   # nx, ny, nz
    h = (0.3, 0.35, 0.5)
    m = (2, 3, 1)
    z, y, x = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    phase = 2 * math.pi * (m[0] * x / n[0] + m[1] * y / n[1] + m[2] * z / n[2])
    u = np.cos(phase)
    lam = sum(4.0 * math.sin(math.pi * m[d] / n[d]) ** 2 / h[d] ** 2 for d in range(3))
    for c in (1.0, 7.5):
        Au = O.apply_A(u, np.full(u.shape, c), h)
        assert np.abs(Au + c * lam * u).max() < 1e-11 * c * lam
        # the vacuum solve inverts the uniform operator on this mode
        assert np.abs(O.vacuum_solve(u, h) + u / lam).max() < 1e-13 * (1 / lam) * 1e2


def test_vacuum_solve_inverts_vacuum_operator():
    h = (0.2, 0.3, 0.25)
    rng = np.random.default_rng(5)
    r = rng.normal(size=(12, 9, 10))
    psi = O.vacuum_solve(r, h)
    assert abs(psi.mean()) < 1e-14
    back = O.apply_A(psi, np.ones_like(r), h)
    assert np.abs(back - (r - r.mean())).max() < 1e-11 * np.abs(r).max()


# ---------------------------------------------------------------- full solve

def test_solve_matches_dense_bordered_direct_solve():
    shape = (8, 8, 8)
    h = (0.3, 0.4, 0.5)
    eps, rho = _rand_case(shape, 11)
    N = rho.size
    A = np.empty((N, N))
    for c in range(N):
        e = np.zeros(N)
        e[c] = 1.0
        A[:, c] = O.apply_A(e.reshape(shape), eps, h).ravel()
    K = np.zeros((N + 1, N + 1))
    K[:N, :N] = A
    K[:N, N] = 1.0
    K[N, :N] = 1.0
    rhs = np.zeros(N + 1)
    rhs[:N] = -FOUR_PI * (rho - rho.mean()).ravel()
    ref = np.linalg.solve(K, rhs)[:N].reshape(shape)
    phi, info = O.solve(rho, eps, h, tol=1e-13, return_info=True)
    assert info["rel_res"] <= 1e-13
    assert np.abs(phi - ref).max() <= 1e-10 * np.abs(ref).max()


def _planar_exact(eps_z, rho_z, hz):
    """Discrete planar solution by integrating the flux (independent of A):
    F_{k+1/2} = C + hz sum_{j<=k} b_j,  phi_{k+1} - phi_k = hz F_{k+1/2} / eps_{k+1/2},
    C fixed by periodicity sum_k F_{k+1/2} / eps_{k+1/2} = 0, then zero mean."""
    nz = len(eps_z)
    b = -FOUR_PI * (rho_z - rho_z.mean())
    ef = 0.5 * (eps_z + np.roll(eps_z, -1))
    S = hz * np.cumsum(b)
    C = -np.sum(S / ef) / np.sum(1.0 / ef)
    F = C + S
    dphi = hz * F / ef
    phi = np.concatenate([[0.0], np.cumsum(dphi)[:-1]])
    return phi - phi.mean()


def test_solve_planar_problem_matches_flux_integration():
    w = W.tanh_box(n=(4, 4, 64))
    eps = w.eps_grid()
    z = np.arange(64) * w.h[2]
    rho_z = np.exp(-((z - 3.0) / 0.7) ** 2) - 0.5 * np.exp(-((z - 12.0) / 1.1) ** 2)
    rho = np.broadcast_to(rho_z[:, None, None], eps.shape).copy()
    phi = O.solve(rho, eps, w.h, tol=1e-13)
    ref = _planar_exact(eps[:, 0, 0], rho_z, w.h[2])
    assert np.abs(phi[:, 2, 1] - ref).max() <= 1e-10 * np.abs(ref).max()


def test_solve_manufactured_solution_second_order():
    L = (6.0, 7.0, 8.0)
    errs = []
    for nn in (8, 16, 32):
        n = (nn, nn, nn)
        h = tuple(L[d] / n[d] for d in range(3))
        z, y, x = np.meshgrid(np.arange(nn) * h[2], np.arange(nn) * h[1], np.arange(nn) * h[0], indexing="ij")
        a = [2 * math.pi / L[d] for d in range(3)]
        sx, sy, sz = np.sin(a[0] * x), np.sin(a[1] * y), np.sin(a[2] * z)
        cx, cy, cz = np.cos(a[0] * x), np.cos(a[1] * y), np.cos(a[2] * z)
        phi_s = sx * sy * sz
        eps_s = 1.0 + 38.0 * (1.0 + cx * cy * cz)
        # grad eps . grad phi + eps lap phi
        ge = (-38 * a[0] * sx * cy * cz, -38 * a[1] * cx * sy * cz, -38 * a[2] * cx * cy * sz)
        gp = (a[0] * cx * sy * sz, a[1] * sx * cy * sz, a[2] * sx * sy * cz)
        lap = -(a[0] ** 2 + a[1] ** 2 + a[2] ** 2) * phi_s
        div = ge[0] * gp[0] + ge[1] * gp[1] + ge[2] * gp[2] + eps_s * lap
        rho = -div / FOUR_PI
        phi = O.solve(rho, eps_s, h, tol=1e-12)
        errs.append(np.abs(phi - phi_s).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 < r1 < 4.8 and 3.6 < r2 < 4.4, errs


def _continuum_energy(w, eps_c):
    """E = (2 pi / (Omega eps)) sum_{G != 0} |S(G)|^2 / G^2 with
    S(G) = sum_j q_j exp(-G^2 sigma^2 / 2) exp(-i G.R_j): Gaussians in a uniform
    dielectric, the G-space form of the vacuum Hartree energy (App. B, Eq. 24)."""
    L = np.array(w.L)
    Om = float(np.prod(L))
    M = 40
    m = np.arange(-M, M + 1)
    Gx, Gy, Gz = np.meshgrid(2 * math.pi * m / L[0], 2 * math.pi * m / L[1], 2 * math.pi * m / L[2], indexing="ij")
    G2 = Gx ** 2 + Gy ** 2 + Gz ** 2
    S = np.zeros(G2.shape, dtype=complex)
    for j in range(len(w.q)):
        S += w.q[j] * np.exp(-0.5 * G2 * w.sigma[j] ** 2) * np.exp(
            -1j * (Gx * w.xyz[j, 0] + Gy * w.xyz[j, 1] + Gz * w.xyz[j, 2]))
    G2[M, M, M] = 1.0
    S[M, M, M] = 0.0
    return 2 * math.pi / (Om * eps_c) * float(np.sum(np.abs(S) ** 2 / G2))


def test_gaussians_in_uniform_dielectric_converge_to_continuum():
    eps_c = 3.0
    errs = []
    for n in ((16, 16, 32), (32, 32, 64), (64, 64, 128)):
        w = W.tanh_box(n=n)
        rho = O.rho_gauss(w.n, w.L, w.xyz, w.q, w.sigma)
        phi = O.solve(rho, np.full(rho.shape, eps_c), w.h, tol=1e-13)
        errs.append(O.energy(rho, phi, w.h))
    Ec = _continuum_energy(W.tanh_box(), eps_c)
    e = [abs(x - Ec) for x in errs]
    assert e[2] < 0.01 * Ec
    assert 3.4 < e[1] / e[2] < 4.6 and 3.0 < e[0] / e[1] < 5.0, (errs, Ec)


def test_uniform_eps_scaling_and_vacuum():
    w = W.tanh_box(n=(16, 16, 32))
    rho = O.rho_gauss(w.n, w.L, w.xyz, w.q, w.sigma)
    p1 = O.solve(rho, np.ones(rho.shape), w.h, tol=1e-13)
    p7 = O.solve(rho, np.full(rho.shape, 7.0), w.h, tol=1e-13)
    vac = O.vacuum_solve(-FOUR_PI * (rho - rho.mean()), w.h)
    assert np.abs(p1 - vac).max() < 1e-11 * np.abs(vac).max()
    assert np.abs(7.0 * p7 - p1).max() < 1e-11 * np.abs(p1).max()


# ---------------------------------------------------------------- energies

def test_energy_invariants():
    h = (0.3, 0.35, 0.4)
    eps, rho = _rand_case((10, 9, 8), 21)
    phi = O.solve(rho, eps, h, tol=1e-13)
    E = O.energy(rho, phi, h)
    assert E > 0
    assert abs(E - O.energy_eps_form(phi, eps, h)) <= 1e-11 * E
    # variational: F[psi] = h^3 rho.psi + (h^3/8 pi) psi.A psi peaks at phi with value E
    h3 = h[0] * h[1] * h[2]
    rng = np.random.default_rng(4)
    v = rng.normal(size=rho.shape)
    vAv = float(np.sum(v * O.apply_A(v, eps, h)))
    for t in (1e-3, 0.1, 1.0):
        psi = phi + t * v
        F = h3 * float(np.sum(rho * psi)) + h3 / (2 * FOUR_PI) * float(np.sum(psi * O.apply_A(psi, eps, h)))
        assert F < E
        assert abs((F - E) - h3 / (2 * FOUR_PI) * t * t * vAv) <= 1e-7 * abs(E) + 1e-9 * abs(F - E)
    # scaling
    phi2 = O.solve(2.5 * rho, eps, h, tol=1e-13)
    assert abs(O.energy(2.5 * rho, phi2, h) - 6.25 * E) <= 1e-11 * E
    phi3 = O.solve(rho, 3.0 * eps, h, tol=1e-13)
    assert abs(O.energy(rho, phi3, h) - E / 3.0) <= 1e-11 * E
    # reciprocity
    _, rho_b = _rand_case((10, 9, 8), 22)
    phib = O.solve(rho_b, eps, h, tol=1e-13)
    assert abs(np.sum(rho * phib) - np.sum(rho_b * phi)) <= 1e-10 * abs(np.sum(rho * phib))
    # integer-node shifts of every input
    sh = (3, -2, 5)
    rs, es = np.roll(rho, sh, axis=(0, 1, 2)), np.roll(eps, sh, axis=(0, 1, 2))
    ps = O.solve(rs, es, h, tol=1e-13)
    assert abs(O.energy(rs, ps, h) - E) <= 1e-11 * E


def test_eps_gradient_matches_finite_differences():
    h = (0.3, 0.35, 0.4)
    eps, rho = _rand_case((8, 8, 8), 31, eps_hi=20.0)
    phi = O.solve(rho, eps, h, tol=1e-13)
    g = O.eps_gradient(phi, h)
    for node in [(0, 0, 0), (3, 5, 7), (7, 2, 4), (4, 4, 1)]:
        d = 1e-4 * eps[node]
        ep, em = eps.copy(), eps.copy()
        ep[node] += d
        em[node] -= d
        Ep = O.energy(rho, O.solve(rho, ep, h, tol=1e-14, max_iter=4000), h)
        Em = O.energy(rho, O.solve(rho, em, h, tol=1e-14, max_iter=4000), h)
        fd = (Ep - Em) / (2 * d)
        assert abs(fd - g[node]) <= 2e-6 * abs(g[node]), (node, fd, g[node])


# ---------------------------------------------------------------- builders

def test_rho_gaussian_moments():
    w = W.slab(n=(48, 48, 192))
    h3 = float(np.prod(w.h))
    for a in (0, 5, 40):
        rho = O.rho_gauss(w.n, w.L, w.xyz[a:a + 1], np.array([1.0]), w.sigma[a:a + 1])
        assert abs(h3 * rho.sum() - 1.0) < 1e-9
        z, y, x = np.meshgrid(np.arange(w.n[2]) * w.h[2], np.arange(w.n[1]) * w.h[1],
                              np.arange(w.n[0]) * w.h[0], indexing="ij")
        d = [x - w.xyz[a, 0], y - w.xyz[a, 1], z - w.xyz[a, 2]]
        d = [di - Ld * np.round(di / Ld) for di, Ld in zip(d, w.L)]
        first = [h3 * float(np.sum(rho * di)) for di in d]
        second = h3 * float(np.sum(rho * (d[0] ** 2 + d[1] ** 2 + d[2] ** 2)))
        assert max(abs(f) for f in first) < 1e-8
        assert abs(second - 3.0 * w.sigma[a] ** 2) < 1e-6


def test_eps_switch_values():
    n = (40, 40, 40)
    L = (10.0, 10.0, 10.0)
    hx = L[0] / n[0]
    xyz = np.array([[20 * hx, 20 * hx, 20 * hx]])
    radius = np.array([8 * hx])
    p = dict(eps_inf=78.36, delta=0.3, exclusion=0, z_lim=0.0, delta_z=0.3)
    eps = O.eps_erf(n, L, xyz, radius, p)
    assert abs(eps[20, 20, 28] - (1.0 + 77.36 / 2)) < 1e-12   # at the radius: s = 1/2
    assert abs(eps[20, 20, 20] - 1.0) < 1e-12                  # centre
    assert abs(eps[0, 0, 0] - 78.36) < 1e-12                    # far away
    assert eps.min() >= 1.0 and eps.max() <= 78.36 + 1e-12
    # exclusion: below a buried atom the permittivity is 1 in the whole plane
    pe = dict(p, exclusion=1, z_lim=3.0)
    xyz2 = np.array([[20 * hx, 20 * hx, 20 * hx], [5.0, 5.0, 2.5]])   # the second one is buried
    eps2 = O.eps_erf(n, L, xyz2, np.array([8 * hx, 1.0]), pe)
    zc = int((2.5 - 6 * 0.3) / hx)
    assert zc >= 2 and np.abs(eps2[:zc + 1] - 1.0).max() < 1e-12
    # well above the buried atom and its switch nothing changes
    assert np.abs(eps2[24:] - eps[24:]).max() < 1e-9
    # without the exclusion rule the same two atoms leave solvent below z = 0.7
    eps3 = O.eps_erf(n, L, xyz2, np.array([8 * hx, 1.0]), p)
    assert eps3[:zc + 1].max() > 78.0


def test_exclusive_products_match_direct_products():
    from oracle.atoms import _exclusive_products
    rng = np.random.default_rng(0)
    f = rng.uniform(0, 1, size=(6, 5))
    f[2, 1] = 0.0
    f[4, 3] = 0.0
    P = _exclusive_products(f)
    for i in range(6):
        ref = np.prod(np.delete(f, i, axis=0), axis=0)
        assert np.allclose(P[i], ref, rtol=1e-15, atol=0)


# ---------------------------------------------------------------- forces

def _energy_of(w, xyz, tol=1e-13):
    eps = O.eps_erf(w.n, w.L, xyz, w.radius, w.eps_params)
    rho = O.rho_gauss(w.n, w.L, xyz, w.q, w.sigma)
    phi = O.solve(rho, eps, w.h, tol=tol, max_iter=4000)
    return O.energy(rho, phi, w.h), eps, rho, phi


@pytest.mark.parametrize("exclusion", [False, True])
def test_forces_match_finite_differences(exclusion):
    w = W.slab(n=(24, 24, 64), exclusion=exclusion)
    E, eps, rho, phi = _energy_of(w, w.xyz)
    g = O.eps_gradient(phi, w.h)
    F = O.forces(w.n, w.L, w.xyz, w.radius, w.q, w.sigma, w.eps_params, phi, g)
    d = 1e-4
    atoms = [3, 30, 60]
    scale = np.abs(F).max()
    for a in atoms:
        for c in range(3):
            xp, xm = w.xyz.copy(), w.xyz.copy()
            xp[a, c] += d
            xm[a, c] -= d
            fd = (_energy_of(w, xp)[0] - _energy_of(w, xm)[0]) / (2 * d)
            assert abs(fd - F[a, c]) <= 2e-6 * scale, (a, c, fd, F[a, c])


def test_dense_derivative_helpers_agree_with_forces():
    w = W.slab(n=(16, 16, 48), exclusion=True)
    E, eps, rho, phi = _energy_of(w, w.xyz, tol=1e-12)
    g = O.eps_gradient(phi, w.h)
    F = O.forces(w.n, w.L, w.xyz, w.radius, w.q, w.sigma, w.eps_params, phi, g)
    h3 = float(np.prod(w.h))
    for a in (0, 17, 65):
        de = O.deps_dR_dense(w.n, w.L, w.xyz, w.radius, w.eps_params, a)
        dr = O.drho_dR_dense(w.n, w.L, w.xyz, w.q, w.sigma, a)
        ref = [float(np.sum(g * de[c]) + h3 * np.sum(phi * dr[c])) for c in range(3)]
        assert np.allclose(F[a], ref, rtol=1e-10, atol=1e-12 * np.abs(F).max())


# ---------------------------------------------------------------- one-pass split

def test_one_pass_split_reduces_to_vacuum_when_eps_is_one():
    w = W.tanh_box(n=(16, 16, 32))
    rho = O.rho_gauss(w.n, w.L, w.xyz, w.q, w.sigma)
    ones = np.ones(rho.shape)
    k0, k1 = W.wet_planes(w.n[2], w.L[2], w.z_wet)
    phiA = O.one_pass_split(rho, ones, w.h, k0, k1)
    ref = O.vacuum_solve(-FOUR_PI * (rho - rho.mean()), w.h)
    assert np.abs(phiA - ref).max() < 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("nz,k0,k1", [(10, 2, 8), (10, 8, 13)])
def test_dirichlet_laplace_solve_inverts_the_slab_laplacian(nz, k0, k1):
    # -L u = v on the slab with u = 0 on every plane outside it (the wrapped
    # slab of the second case runs through plane 0), L from apply_A with eps = 1
    from oracle.split import dirichlet_laplace_solve
    h = (0.4, 0.5, 0.3)
    planes = np.arange(k0, k1) % nz
    v = np.random.default_rng(3).normal(size=(len(planes), 6, 4))
    u = dirichlet_laplace_solve(v, h)
    full = np.zeros((nz, 6, 4))
    full[planes] = u
    back = -O.apply_A(full, np.ones_like(full), h)[planes]
    assert np.abs(back - v).max() <= 1e-12 * np.abs(v).max()


@pytest.mark.parametrize("k0,k1", [(3, 7), (6, 11)])
def test_one_pass_split_matches_a_dense_solve(k0, k1):
    # steps 1-3 of the split written out with a dense matrix on a 4 x 5 x 8 grid:
    # phi_vac from the FFT, then the wet unknowns from the dense Dirichlet system
    # (columns of -A restricted to W), then the zero-mean shift
    n, h = (4, 5, 8), (0.5, 0.4, 0.45)
    rng = np.random.default_rng(11)
    eps = rng.uniform(1.0, 30.0, size=(n[2], n[1], n[0]))
    rho = rng.normal(size=eps.shape)
    b = -FOUR_PI * (rho - rho.mean())
    phi_vac = O.vacuum_solve(b, h)
    wet = np.zeros(n[2], dtype=bool)
    wet[np.arange(k0, k1) % n[2]] = True
    idx = np.flatnonzero(np.broadcast_to(wet[:, None, None], eps.shape))
    cols = []
    for c in idx:
        e = np.zeros(eps.size)
        e[c] = 1.0
        cols.append(-O.apply_A(e.reshape(eps.shape), eps, h).ravel()[idx])
    Aw = np.array(cols).T
    dry = phi_vac.ravel().copy()
    dry[idx] = 0.0
    rhs = -(b.ravel() - O.apply_A(dry.reshape(eps.shape), eps, h).ravel())[idx]
    phi = phi_vac.ravel().copy()
    phi[idx] = np.linalg.solve(Aw, rhs)
    ref = (phi - phi.mean()).reshape(eps.shape)
    got = O.one_pass_split(rho, eps, h, k0, k1)
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()
