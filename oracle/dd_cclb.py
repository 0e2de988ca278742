"""FP64 reference oracle of the DD-CCLB time step (arXiv 2311.10314).

TEST INFRASTRUCTURE. Only tests/, __graft_entry__.smoke() and the cpu_baseline
leg of bench.py may import or run this module. The product path (the HIP
library and its binding) never calls it and shares no code with it.

What it computes: one time step of the diffuse-domain consistent and
conservative lattice Boltzmann method of Section 3, for N phases, in plain
numpy float64, each stage a whole-grid sweep in the order the scheme needs:

  moments (phi C_i = sum_p f^i_p)                 Section 3, moment recovery
  finite-difference gradients / div(phi grad C)   eq. (2.14) and Section 3
  chemical potential phi mu_i                     eq. (2.14)
  mobility M_ij, source vector S_i, flux m^C      eqs. (2.5), (3.7), Sec. 2.2
  force F and velocity u                          eq. (3.13), moment recovery
  pressure                                        eq. (19)
  equilibria and sources                          eqs. (3.5), (3.6), (3.8)-(3.12)
  collision Lambda = H^-1 S H                     eqs. (3.1)-(3.4)
  streaming (pull, periodic)                      eqs. (3.1), (3.2) left sides

Readings where the paper is silent or garbled are the same as the library's;
each is marked "Reading:" below where it is applied.
Notation: psi is the paper's smooth characteristic function phi (fluid 1,
solid 0); phi C_i is written psiC; lattice units dx = dt = c = 1, c_s^2 = d0.

Grid arrays are (ny, nx) in 2D and (nz, ny, nx) in 3D; vector component a
(0 = x, 1 = y, 2 = z) runs along array axis -1 - a. All walls are embedded
through psi and the box is periodic in every direction.
"""
import numpy as np

from .lattices import Lattice, stencil_lattice

RATE_KEYS = ("0", "1", "21", "22", "3", "4")


# --------------------------------------------------------------------------
# Array helpers. The grid functions below take numpy float64 arrays; they
# also take torch float64 CPU tensors, with the same arithmetic, so that
# oracle.adjoint can differentiate this very step by reverse-mode automatic
# differentiation. Constants (lattice tables, parameters) stay numpy.
# --------------------------------------------------------------------------
def _is_torch(a):
    return type(a).__module__.split(".")[0] == "torch"


def zeros(shape, like):
    """float64 zeros of `shape`, a torch tensor if `like` is one."""
    if _is_torch(like):
        return like.new_zeros(tuple(int(v) for v in shape))
    return np.zeros(shape)


def stack(arrays):
    arrays = list(arrays)
    if _is_torch(arrays[0]):
        import torch
        return torch.stack(arrays)
    return np.array(arrays)


def as_f64(a):
    """A float64 grid array: torch tensors pass through, the rest goes to
    numpy."""
    return a if _is_torch(a) else np.array(a, dtype=np.float64)


def _roll(a, shift, axis):
    if _is_torch(a):
        import torch
        return torch.roll(a, shift, dims=axis)
    return np.roll(a, shift, axis=axis)


def floor_at(a, m):
    """max(a, m) elementwise."""
    if _is_torch(a):
        import torch
        return torch.clamp(a, min=m)
    return np.maximum(a, m)


def vector_norm(v):
    """|v| over the first axis. Its derivative at v = 0 is taken as 0 (the
    torch path guards the square root there)."""
    s = (v ** 2).sum(axis=0)
    if _is_torch(v):
        import torch
        pos = s > 0
        return torch.where(pos, torch.sqrt(torch.where(pos, s,
                                                       torch.ones_like(s))),
                           torch.zeros_like(s))
    return np.sqrt(s)


def _apply(mat, x):
    """sum_q mat[k, q] x[q] for a constant (Q, Q) matrix and x of shape
    (Q,) + grid."""
    if _is_torch(x):
        import torch
        return torch.tensordot(torch.as_tensor(mat, dtype=x.dtype), x,
                               dims=([1], [0]))
    return np.tensordot(mat, x, axes=(1, 0))


# --------------------------------------------------------------------------
# Parameters
# --------------------------------------------------------------------------
class Params:
    """Physical and numerical parameters in lattice units.

    sigma: N x N symmetric surface tensions, zero diagonal (Section 2.1).
    rho, nu: per-phase density and kinematic viscosity (linear mixing, 2.2).
    m0: mobility of eq. (2.5); eta_i derived from eq. (17) unless given.
    eps: fluid-fluid interface width; eps0: diffuse-domain layer thickness.
    lam: penalty coefficient of (1 - psi) u (eq. 2.13c); default 1/eps0^3.
    accel, force: body acceleration a and body force density G (force psi
      rho a + psi G).
    s_f: relaxation rates of the phase sets; s_g: those of the flow set
      ('21' and '22' of the flow set always come from nu(x) by eq. (16)).
    """

    def __init__(self, *, dim, lattice_f, lattice_g, d0, eps, m0, sigma, rho,
                 nu, eps0=None, lam=None, rho0=1.0, psi_min=1e-30, s_f=None,
                 s_g=None, eta=None, accel=None, force=None):
        self.dim = int(dim)
        self.sigma = np.array(sigma, dtype=np.float64)
        self.N = self.sigma.shape[0]
        self.rho = np.array(rho, dtype=np.float64)
        self.nu = np.array(nu, dtype=np.float64)
        self.d0 = float(d0)
        self.cs2 = float(d0)
        self.eps = float(eps)
        self.m0 = float(m0)
        if lam is None:
            lam = 1.0 / float(eps0) ** 3          # Reading: lambda = 1/eps0^3
        self.lam = float(lam)
        self.rho0 = float(rho0)
        self.psi_min = float(psi_min)
        sf = {"0": 1.0, "1": 10.0 / 19.0, "21": 1.2, "22": 1.2, "3": 1.2,
              "4": 1.2}
        sg = {"0": 1.0, "1": 1.2, "3": 1.2, "4": 1.2}
        sf.update(s_f or {})
        sg.update(s_g or {})
        self.s_f = sf
        self.s_g = sg
        self.lat_f = Lattice(lattice_f, d0)
        self.lat_g = Lattice(lattice_g, d0)
        assert self.lat_f.d == self.dim and self.lat_g.d == self.dim
        # beta_ij and kappa_ij, Section 2.1. Reading: beta_ij = 3 sigma_ij/eps
        # (printed as 3 eps/sigma_ij; only this form gives beta_ii = 0 and the
        # two-phase tanh profile of width eps).
        self.beta = 3.0 * self.sigma / self.eps
        # eq. (17): m0 = (1/s1 - 1/2) eta_i c_s^2 dt
        if eta is None:
            eta = self.m0 / ((1.0 / self.s_f["1"] - 0.5) * self.cs2)
        self.eta = np.broadcast_to(np.array(eta, dtype=np.float64),
                                   (self.N,)).copy()
        self.accel = np.zeros(self.dim) if accel is None else \
            np.array(accel, dtype=np.float64)
        self.force = np.zeros(self.dim) if force is None else \
            np.array(force, dtype=np.float64)
        # eq. (19) constants. K = w0 / (1 - d0) equals the printed K for both
        # the 2D (1 - d0) and the 3D (1 - 2 d0) lattices; the printed H
        # factor is (1 - 2 d0) in 2D and (3 - 7 d0)/2 in 3D (H also carries
        # (s21 - 2), applied per node).
        w0 = self.lat_g.w[0]
        self.K = w0 / (1.0 - self.d0)
        self.Hfac = (1.0 - 2.0 * self.d0) if self.dim == 2 else \
            (3.0 - 7.0 * self.d0) / 2.0


# --------------------------------------------------------------------------
# Periodic finite differences (Reading: the paper gives no stencils; a fixed
# isotropic stencil, D2Q9 or D3Q19 weights at d0 = 1/3, is used)
# --------------------------------------------------------------------------
def shifted(field, c):
    """field(x + c) on the periodic grid; the last len(c) axes are spatial."""
    out = field
    for a, ca in enumerate(c):
        if ca != 0:
            out = _roll(out, -int(ca), -1 - a)
    return out


def grad(field, d):
    """Central isotropic gradient: sum_p w_p c_p field(x + c_p) / c_s^2.
    Returns shape (d,) + field.shape."""
    cst, wst, cs2 = stencil_lattice(d)
    out = zeros((d,) + tuple(field.shape), field)
    for p in range(1, len(wst)):
        fs = shifted(field, cst[p])
        for a in range(d):
            if cst[p][a] != 0:
                out[a] += wst[p] * cst[p][a] * fs
    return out / cs2


def div_psi_grad(psi, C, d):
    """Conservative div(psi grad C), the term of eq. (2.14):
    sum_p w_p [psi(x + c_p) + psi(x)] [C(x + c_p) - C(x)] / c_s^2."""
    cst, wst, cs2 = stencil_lattice(d)
    out = zeros(C.shape, C)
    for p in range(1, len(wst)):
        out += wst[p] * (shifted(psi, cst[p]) + psi) * (shifted(C, cst[p]) - C)
    return out / cs2


def div_tensor(T, d):
    """(div T)_b = sum_a d_a T_ab for T of shape (d, d) + grid."""
    out = zeros((d,) + tuple(T.shape[2:]), T)
    for b in range(d):
        out[b] = sum(grad(T[a, b], d)[a] for a in range(d))
    return out


# --------------------------------------------------------------------------
# Static geometry
# --------------------------------------------------------------------------
def pair_cosines(prm, cos_theta_iN, shape):
    """eq. (2.9): cos th_ij = (s_iN cos th_iN - s_jN cos th_jN) / s_ij for
    every pair i != j, from the N - 1 angles theta_iN measured against the
    N-th phase (its own entry cos th_NN is absent, sigma_NN = 0)."""
    N = prm.N
    cos_theta_iN = as_f64(cos_theta_iN)
    ct = zeros((N,) + tuple(shape), cos_theta_iN)
    if N > 1:
        ct[:N - 1] = cos_theta_iN.reshape((N - 1,) + tuple(shape))
    sg = prm.sigma
    out = zeros((N, N) + tuple(shape), cos_theta_iN)
    for i in range(N):
        for j in range(N):
            if i != j:
                out[i, j] = (sg[i, N - 1] * ct[i] - sg[j, N - 1] * ct[j]) \
                    / sg[i, j]
    return out


class Geometry:
    """psi, psi_hat = max(psi, psi_min), grad psi, |grad psi| and, per wall,
    the contact-angle cosines cos theta_jq of eq. (2.9) with the |grad psi_k|
    that weights them in the wetting term of eq. (2.14).

    One wall: psi and its angles. Several walls (Section 4.5): `walls` is a
    list of (psi_k, cos_theta_iN^k); then psi = prod_k psi_k and the wetting
    term sums cos theta^k_jq |grad psi_k| over the walls."""

    def __init__(self, prm, psi, cos_theta_iN, walls=None):
        d = prm.dim
        if walls is None:
            walls = [(psi, cos_theta_iN)]
            self.psi = as_f64(psi)
        else:
            self.psi = as_f64(walls[0][0])
            for psi_k, _ in walls[1:]:
                self.psi = self.psi * as_f64(psi_k)
        # Reading: division by psi uses psi_hat = max(psi, psi_min).
        self.psi_hat = floor_at(self.psi, prm.psi_min)
        self.grad_psi = grad(self.psi, d)
        self.abs_grad_psi = vector_norm(self.grad_psi)
        self.walls = []
        for psi_k, ct_k in walls:
            g = grad(as_f64(psi_k), d)
            self.walls.append((pair_cosines(prm, ct_k, self.psi.shape),
                               vector_norm(g)))
        self.cos_theta = self.walls[0][0]


# --------------------------------------------------------------------------
# Physics pieces
# --------------------------------------------------------------------------
def g_prime(C):
    """g(C) = C^2 (C - 1)^2  =>  g'(C) = 2 C (C - 1)(2 C - 1)."""
    return 2.0 * C * (C - 1.0) * (2.0 * C - 1.0)


def chemical_potential(prm, geo, C, L):
    """phi mu_i of eq. (2.14): bulk + gradient (L_j = div(psi grad C_j)) +
    wetting term sum_j 3 sigma_ij sum_{q != j} cos th_jq C_j C_q |grad psi|,
    summed over the walls (cos th^k_jq |grad psi_k|, Section 4.5)."""
    N = prm.N
    psi = geo.psi
    out = zeros(C.shape, C)
    for i in range(N):
        acc = zeros(psi.shape, C)
        for j in range(N):
            acc += 2.0 * prm.beta[i, j] * psi * (g_prime(C[i])
                                                 - g_prime(C[i] + C[j]))
        for j in range(N):
            acc += 0.75 * prm.eps * prm.sigma[i, j] * L[j]
        total = zeros(psi.shape, C)
        for cos_theta, abs_grad_psi_k in geo.walls:
            wet = zeros(psi.shape, C)
            for j in range(N):
                inner = zeros(psi.shape, C)
                for q in range(N):
                    if q != j:
                        inner += cos_theta[j, q] * C[j] * C[q]
                wet += 3.0 * prm.sigma[i, j] * inner
            total += wet * abs_grad_psi_k
        out[i] = acc + total
    return out


def mobility(prm, C):
    """eq. (2.5): M_ij = -m0 C_i C_j (i != j), M_ii = -sum_{j != i} M_ij."""
    N = prm.N
    M = zeros((N, N) + tuple(C.shape[1:]), C)
    for i in range(N):
        for j in range(N):
            if i != j:
                M[i, j] = -prm.m0 * C[i] * C[j]
    for i in range(N):
        M[i, i] = -sum(M[i, j] for j in range(N) if j != i)
    return M


def source_vector(prm, psi, M, grad_mu):
    """eq. (3.7): S_i = (psi M_ii - psi m0)/m0 grad mu_i
                       + sum_{j != i} psi M_ij / m0 grad mu_j."""
    N = prm.N
    S = zeros(grad_mu.shape, grad_mu)
    for i in range(N):
        S[i] = (psi * M[i, i] - psi * prm.m0) / prm.m0 * grad_mu[i]
        for j in range(N):
            if j != i:
                S[i] += psi * M[i, j] / prm.m0 * grad_mu[j]
    return S


def mass_flux(prm, M, grad_mu):
    """Section 2.2: m^C = -sum_ij rho_i M_ij grad mu_j."""
    N = prm.N
    out = zeros(grad_mu.shape[1:], grad_mu)
    for i in range(N):
        for j in range(N):
            out -= prm.rho[i] * M[i, j] * grad_mu[j]
    return out


def flow_rates(prm, nu):
    """eq. (16): nu = (1/s21 - 1/2)(c^2 - c_s^2)/2 dt = (1/s22 - 1/2) c_s^2 dt,
    solved for the per-node rates s21, s22."""
    s21 = 1.0 / (2.0 * nu / (1.0 - prm.cs2) + 0.5)
    s22 = 1.0 / (nu / prm.cs2 + 0.5)
    return s21, s22


def hermite2_expansion(lat, A):
    """Second-order Hermite expansion used by s_p and G_p (eqs. 3.10, 3.11):
    sum_a A_aa (c_pa^2 - c_s^2)/(c^2 c_s^2 - c_s^4)
      + sum over unordered pairs a < b of A_ab c_pa c_pb / c_s^4.
    Reading: the off-diagonal sum has one term per unordered pair (the only
    form that gives the second-moment identity (B.5d)).
    Returns a (Q,) + grid array (without the weight w_p)."""
    cs2 = lat.cs2
    d = lat.d
    out = zeros((lat.Q,) + tuple(A.shape[2:]), A)
    for p in range(lat.Q):
        c = lat.c[p]
        for a in range(d):
            out[p] += A[a, a] * (c[a] * c[a] - cs2) / (cs2 - cs2 * cs2)
        for a in range(d):
            for b in range(a + 1, d):
                out[p] += A[a, b] * (c[a] * c[b]) / (cs2 * cs2)
    return out


def f_equilibrium(lat, psiC_i, psimu_i, X_i, eta_i):
    """eq. (3.5): p = 0: (w_0 - 1) eta phi mu + phi C;
                  p != 0: w_p eta phi mu + w_p c_p . (phi C u) / c_s^2."""
    cs2 = lat.cs2
    out = zeros((lat.Q,) + tuple(psiC_i.shape), psiC_i)
    for p in range(lat.Q):
        cu = sum(lat.c[p][a] * X_i[a] for a in range(lat.d))
        if p == 0:
            out[p] = (lat.w[0] - 1.0) * eta_i * psimu_i + psiC_i
        else:
            out[p] = lat.w[p] * eta_i * psimu_i + lat.w[p] * cu / cs2
    return out


def f_source(lat, V_i):
    """eq. (3.6): F^i_p = w_p c_p . V / c_s^2 with
    V = d_t(phi C_i u) + c_s^2 eta_i (mu_i grad phi - S_i)."""
    out = zeros((lat.Q,) + tuple(V_i.shape[1:]), V_i)
    for p in range(lat.Q):
        out[p] = lat.w[p] * sum(lat.c[p][a] * V_i[a]
                                for a in range(lat.d)) / lat.cs2
    return out


def g_equilibrium(lat, psiP, rho0, psirho, u, Y):
    """eqs. (3.8), (3.11): g^eq_0 = (w_0 - 1) phi P / c_s^2 + rho0 + s_0,
    g^eq_p = w_p phi P / c_s^2 + s_p, with s_p = w_p [c_p . phi rho u / c_s^2
    + Hermite-2 expansion of A = phi rho u u + (phi m^C u + phi u m^C)/2].
    Y is the symmetric part (phi m^C u + phi u m^C)/2."""
    d = lat.d
    cs2 = lat.cs2
    A = zeros((d, d) + tuple(psiP.shape), psiP)
    for a in range(d):
        for b in range(d):
            A[a, b] = psirho * u[a] * u[b] + Y[a, b]
    h2 = hermite2_expansion(lat, A)
    out = zeros((lat.Q,) + tuple(psiP.shape), psiP)
    for p in range(lat.Q):
        cj = sum(lat.c[p][a] * psirho * u[a] for a in range(d))
        s_p = lat.w[p] * (cj / cs2 + h2[p])
        if p == 0:
            out[p] = (lat.w[0] - 1.0) * psiP / cs2 + rho0 + s_p
        else:
            out[p] = lat.w[p] * psiP / cs2 + s_p
    return out


def equilibrium_s0(lat, psirho, u, Y):
    """The p = 0 component s_0 of eq. (3.11), which also enters eq. (19):
    s_0 = w_0 sum_a A_aa (0 - c_s^2)/(c^2 c_s^2 - c_s^4)."""
    trA = sum(psirho * u[a] * u[a] + Y[a, a] for a in range(lat.d))
    return -lat.w[0] * trA / (1.0 - lat.cs2)


def m2g_tensor(lat, dtY, u, grad_psirho):
    """M^{2G} of eq. (3.12):
    d_t (phi m^C u + phi u m^C)/2 + c_s^2 [u grad(phi rho) + grad(phi rho) u]
      + (c^2 - 3 c_s^2) u . grad(phi rho) I.
    Reading: the last term is the scalar u . grad(phi rho) times the identity,
    as printed; Appendix C's pressure recipe reproduces the printed constants
    of eq. (19) with exactly this form."""
    d = lat.d
    cs2 = lat.cs2
    udotb = sum(u[a] * grad_psirho[a] for a in range(d))
    M = zeros(dtY.shape, dtY)
    for a in range(d):
        for b in range(d):
            M[a, b] = dtY[a, b] + cs2 * (u[a] * grad_psirho[b]
                                         + grad_psirho[a] * u[b])
        M[a, a] += (1.0 - 3.0 * cs2) * udotb
    return M


def g_source(lat, psi, u, grad_rho, F, M2G):
    """eq. (3.10): G_p = w_p [phi u . grad rho + c_p . F / c_s^2
                          + Hermite-2 expansion of M^{2G}]."""
    d = lat.d
    a0 = psi * sum(u[a] * grad_rho[a] for a in range(d))
    h2 = hermite2_expansion(lat, M2G)
    out = zeros((lat.Q,) + tuple(psi.shape), u)
    for p in range(lat.Q):
        cF = sum(lat.c[p][a] * F[a] for a in range(d))
        out[p] = lat.w[p] * (a0 + cF / lat.cs2 + h2[p])
    return out


def collide(lat, pop, eq, src, rates):
    """eqs. (3.1)-(3.4): f* = f - Lambda (f - f^eq) + dt (I - Lambda/2) F with
    Lambda = H^-1 S H; S may vary per node (rates: list of Q scalars/arrays)."""
    m_ne = _apply(lat.H, pop - eq)
    m_src = _apply(lat.H, src)
    mstar = zeros(m_ne.shape, m_ne)
    for k in range(lat.Q):
        s = rates[k]
        mstar[k] = s * m_ne[k] - (1.0 - 0.5 * s) * m_src[k]
    return pop - _apply(lat.Hinv, mstar)


def stream(lat, post):
    """Pull streaming, periodic: f_p(x, t + dt) = f*_p(x - c_p, t)."""
    out = zeros(post.shape, post)
    for p in range(lat.Q):
        out[p] = shifted(post[p], -lat.c[p])
    return out


# --------------------------------------------------------------------------
# State and the step
# --------------------------------------------------------------------------
class State:
    """Populations f (N, Qf, grid), g (Qg, grid) and the previous-step values
    kept for the time derivatives and the lagged terms:
    X = phi C_i u (N, d, grid), Y = (phi m^C u + phi u m^C)/2 (d, d, grid),
    P (grid), T = (phi m^C u - phi u m^C)/2 (d, d, grid)."""

    def __init__(self, f, g, X, Y, P, T):
        self.f, self.g, self.X, self.Y, self.P, self.T = f, g, X, Y, P, T

    def copy(self):
        return State(self.f.copy(), self.g.copy(), self.X.copy(),
                     self.Y.copy(), self.P.copy(), self.T.copy())


def volume_fractions(prm, geo, psiC):
    """C_i from the recovered moments phi C_i.
    Reading: C_i = phi C_i / sum_j phi C_j. In the model sum_j C_j = 1
    (Section 2.1), so sum_j phi C_j = phi and this is the printed
    C_i = phi C_i / phi; taking the sum of the recovered moments as the
    divisor keeps the constraint exact on the lattice and keeps C_i defined
    where phi underflows inside solids. With the printed divisor (floored at
    psi_min) a density-ratio-100 droplet on a wall diverges within 2000
    steps; with this one it stays bounded (test_oracle_physics)."""
    return psiC / floor_at(psiC.sum(axis=0), prm.psi_min)


def _phase_fields(prm, geo, psiC):
    """From phi C_i: C, rho, nu, gradients, phi mu, mu, grad mu, M, S, m^C."""
    d = prm.dim
    N = prm.N
    psi = geo.psi
    C = volume_fractions(prm, geo, psiC)
    rho = sum(prm.rho[i] * C[i] for i in range(N))           # linear mixing
    nu = sum(prm.nu[i] * C[i] for i in range(N))
    psirho = psi * rho
    gradC = stack([grad(C[i], d) for i in range(N)])         # (N, d, grid)
    L = stack([div_psi_grad(psi, C[j], d) for j in range(N)])
    grad_rho = sum(prm.rho[i] * gradC[i] for i in range(N))
    grad_psirho = grad(psirho, d)
    psimu = chemical_potential(prm, geo, C, L)
    mu = psimu / geo.psi_hat
    grad_mu = stack([grad(mu[i], d) for i in range(N)])
    M = mobility(prm, C)
    S = source_vector(prm, psi, M, grad_mu)
    mC = mass_flux(prm, M, grad_mu)
    return dict(C=C, rho=rho, nu=nu, psirho=psirho, gradC=gradC,
                grad_rho=grad_rho, grad_psirho=grad_psirho, psimu=psimu,
                mu=mu, S=S, mC=mC)


def _tensors(psi, mC, u):
    d = u.shape[0]
    Y = zeros((d, d) + tuple(psi.shape), u)
    T = zeros((d, d) + tuple(psi.shape), u)
    for a in range(d):
        for b in range(d):
            Y[a, b] = 0.5 * (psi * mC[a] * u[b] + psi * u[a] * mC[b])
            T[a, b] = 0.5 * (psi * mC[a] * u[b] - psi * u[a] * mC[b])
    return Y, T


def macroscopic(prm, geo, st):
    """Every node quantity of the current time level from the populations
    and the previous-step values (no collision)."""
    d = prm.dim
    N = prm.N
    lat_g = prm.lat_g
    psi = geo.psi
    psiC = st.f.sum(axis=1)                                  # phi C_i = sum_p f^i_p
    q = _phase_fields(prm, geo, psiC)
    psirho = q["psirho"]
    j = stack([sum(lat_g.c[p][a] * st.g[p] for p in range(lat_g.Q))
               for a in range(d)])
    sum_g_moving = st.g[1:].sum(axis=0)
    # eq. (3.13): F = -div T + sum_i phi mu_i grad C_i + P grad phi
    #               - (1 - phi) lam u, plus phi (rho a + G) for a body
    #               acceleration a or a body force density G.
    # Reading: T and P are taken from the previous step (they need u);
    # the penalty is solved implicitly with the velocity recovery below.
    Fp = -div_tensor(st.T, d) + st.P * geo.grad_psi
    for i in range(N):
        Fp += q["psimu"][i] * q["gradC"][i]
    for a in range(d):
        Fp[a] += psirho * prm.accel[a] + psi * prm.force[a]
    # phi rho u = sum_p c_p g_p + F/2 with F = Fp - (1 - phi) lam u
    u = (j + 0.5 * Fp) / (psirho + 0.5 * (1.0 - psi) * prm.lam)
    F = Fp - (1.0 - psi) * prm.lam * u
    X = psiC[:, None] * u[None]                               # phi C_i u
    dtX = X - st.X                                            # Reading: backward difference
    Y, T = _tensors(psi, q["mC"], u)
    dtY = Y - st.Y
    s21, s22 = flow_rates(prm, q["nu"])
    s0eq = equilibrium_s0(lat_g, psirho, u, Y)
    udotgr = sum(u[a] * q["grad_rho"][a] for a in range(d))
    udotgpr = sum(u[a] * q["grad_psirho"][a] for a in range(d))
    trdtY = sum(dtY[a, a] for a in range(d))
    Hc = prm.K * prm.Hfac * (s21 - 2.0)
    sg0 = prm.s_g["0"]
    # eq. (19)
    w0 = lat_g.w[0]
    psiP = prm.cs2 / (1.0 - w0) * (
        sum_g_moving
        + (0.5 + prm.K * (1.0 - prm.d0) * (2.0 - sg0) / (2.0 * sg0))
        * psi * udotgr
        + 0.5 * prm.K * trdtY
        + Hc / s21 * udotgpr
        + s0eq)
    P = psiP / geo.psi_hat
    q.update(psiC=psiC, u=u, F=F, X=X, dtX=dtX, Y=Y, dtY=dtY, T=T, s21=s21,
             s22=s22, psiP=psiP, P=P)
    return q


def step(prm, geo, st):
    """Advance one time step; returns the new State."""
    d = prm.dim
    N = prm.N
    lat_f, lat_g = prm.lat_f, prm.lat_g
    psi = geo.psi
    q = macroscopic(prm, geo, st)
    cs2 = prm.cs2
    rates_f = lat_f.rate_vector(prm.s_f)
    f_new = zeros(st.f.shape, st.f)
    for i in range(N):
        feq = f_equilibrium(lat_f, q["psiC"][i], q["psimu"][i], q["X"][i],
                            prm.eta[i])
        V = q["dtX"][i] + cs2 * prm.eta[i] * (q["mu"][i] * geo.grad_psi
                                              - q["S"][i])
        Fi = f_source(lat_f, V)
        f_new[i] = stream(lat_f, collide(lat_f, st.f[i], feq, Fi, rates_f))
    geq = g_equilibrium(lat_g, q["psiP"], prm.rho0, q["psirho"], q["u"],
                        q["Y"])
    M2G = m2g_tensor(lat_g, q["dtY"], q["u"], q["grad_psirho"])
    G = g_source(lat_g, psi, q["u"], q["grad_rho"], q["F"], M2G)
    rg = dict(prm.s_g)
    rg["21"] = q["s21"]
    rg["22"] = q["s22"]
    g_new = stream(lat_g, collide(lat_g, st.g, geq, G, lat_g.rate_vector(rg)))
    return State(f_new, g_new, q["X"], q["Y"], q["P"], q["T"])


def init_state(prm, geo, C0, u0=None, P0=None):
    """Populations at equilibrium with the given C, u, P (Reading: f = f^eq,
    g = g^eq, and previous-step values equal to the initial ones, so every
    time derivative starts at zero)."""
    d = prm.dim
    N = prm.N
    psi = geo.psi
    shape = psi.shape
    C0 = np.array(C0, dtype=np.float64).reshape((N,) + shape)
    u = np.zeros((d,) + shape) if u0 is None else \
        np.array(u0, dtype=np.float64).reshape((d,) + shape)
    P = np.zeros(shape) if P0 is None else \
        np.array(P0, dtype=np.float64).reshape(shape)
    psiC = psi * C0
    q = _phase_fields(prm, geo, psiC)
    X = psiC[:, None] * u[None]
    Y, T = _tensors(psi, q["mC"], u)
    lat_f, lat_g = prm.lat_f, prm.lat_g
    f = np.empty((N, lat_f.Q) + shape)
    for i in range(N):
        f[i] = f_equilibrium(lat_f, psiC[i], q["psimu"][i], X[i], prm.eta[i])
    g = g_equilibrium(lat_g, psi * P, prm.rho0, q["psirho"], u, Y)
    return State(f, g, X, Y, P.copy(), T)


def moments(prm, geo, st):
    """C_i, u and P of the current time level (no time advance)."""
    q = macroscopic(prm, geo, st)
    return q["C"], q["u"], q["P"]


def mass(st):
    """Per-phase total sum_x sum_p f^i_p."""
    N = st.f.shape[0]
    return np.array([st.f[i].sum() for i in range(N)])


def run(prm, geo, st, nsteps):
    for _ in range(int(nsteps)):
        st = step(prm, geo, st)
    return st
