"""Problem definitions and seeded input generators.

Everything here is input to the solver, not part of it:

* the KL data of the coefficient (eq. (KL-expansion), eq. (int-eigproblem),
  eq. (cov) of Section 2), computed numerically on the mesh with a separable
  Nystrom method;
* nodal right-hand-side values f(x_i) and the lumped load vector h^2 f(x_i)
  (f is deterministic, so only the mean chaos block of the load is non-zero,
  eq. (global-system));
* quantity-of-interest weights, seeded random blocks and the workload
  parameter sets.

Conventions shared by every consumer:

* the unit square carries ``n_e x n_e`` Q1 elements, ``h = 1/n_e``;
* interior nodes ``(ix, iy)``, ``1 <= ix, iy <= n_e - 1``, are numbered
  ``(iy - 1) * (n_e - 1) + (ix - 1)`` (x1 fastest), ``n = (n_e - 1)^2``;
* element ``(ex, ey)``, ``0 <= ex, ey < n_e``, has corners
  ``(ex, ey) .. (ex + 1, ey + 1)``; element arrays are ``[ey, ex]``;
* the coefficient is ``a(x, xi) = theta0 + sigma * sum_k s_k phi_k(x) xi_k``
  with ``s_k = sqrt(lambda_k)`` and ``xi_k`` i.i.d.: standard Gaussian
  (``family = "hermite"``, the default) or uniform on ``[-1, 1]``
  (``family = "legendre"``, the paper's examples; sigma is then the nominal
  coefficient of variation);
* a block of chaos coefficients is stored as an array of shape ``(P, n)``:
  row ``j`` is the nodal vector of chaos coefficient ``j`` (column-major
  ``n x P``, the paper's stacked vector ``[u_0; ...; u_M]``).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from numpy.polynomial import hermite_e, legendre


def n_chaos(M: int, p: int) -> int:
    """Number of chaos polynomials of total degree <= p in M variables."""
    return math.comb(M + p, p)


@dataclass
class Problem:
    name: str
    n_e: int
    M: int
    p: int
    theta0: float
    sigma: float
    L: float
    s: np.ndarray            # (M,) KL amplitudes sqrt(lambda_k)
    phi: np.ndarray          # (M, n_e, n_e) element values of the KL modes, [k, ey, ex]
    f_nodal: np.ndarray      # (n,) f at the interior nodes
    modes: list = field(default_factory=list)  # (i, j) 1D mode pairs of each KL term
    family: str = "hermite"  # distribution of xi and chaos family: "hermite" or "legendre"

    @property
    def n(self) -> int:
        return (self.n_e - 1) ** 2

    @property
    def P(self) -> int:
        return n_chaos(self.M, self.p)

    @property
    def h(self) -> float:
        return 1.0 / self.n_e

    def load_block(self) -> np.ndarray:
        """Right-hand side block F, shape (P, n): row 0 is the lumped load h^2 f(x_i).

        For f = 1 the lumped value equals the exact integral of a Q1 hat
        function (h^2), so the load is exact there.
        """
        F = np.zeros((self.P, self.n))
        F[0] = self.h * self.h * self.f_nodal
        return F

    def element_coefficients(self) -> np.ndarray:
        """KL coefficient fields sigma * s_k * phi_k(e), shape (M, n_e, n_e)."""
        return self.sigma * self.s[:, None, None] * self.phi

    def coefficient_margin(self) -> float:
        """Lower bound of the element chaos matrices theta0 I + sum_k a_k(e) G_k.

        Hermite (exact): by rotation invariance of the Gaussian measure, the
        total-degree-p chaos space is mapped onto itself by orthogonal changes
        of xi, so the extreme eigenvalue of multiplication by
        ``sum_k a_k xi_k`` on it is ``||a||_2`` times the largest zero of
        He_{p+1}. Legendre (a bound): the space lies in the tensor space of
        degree p per variable, where that multiplication has the eigenvalues
        ``sum_k a_k x_k`` over the (p+1)-point Gauss nodes of each variable,
        so ``sum_k |a_k|`` times the largest node bounds it. If the returned
        margin is positive every element matrix is SPD, hence the global SG
        matrix is SPD. Uses only Gauss nodes of library routines.
        """
        if self.M == 0 or self.p == 0:
            return float(self.theta0)
        a = self.element_coefficients()
        if self.family == "legendre":
            xmax = float(np.max(legendre.leggauss(self.p + 1)[0]))
            return float(self.theta0 - xmax * np.abs(a).sum(axis=0).max())
        xmax = float(np.max(hermite_e.hermegauss(self.p + 1)[0]))
        anorm = np.sqrt(np.sum(a * a, axis=0))
        return float(self.theta0 - xmax * anorm.max())


# ---------------------------------------------------------------------------
# KL expansion of the separable exponential covariance (Section 2, eq. (cov))
# ---------------------------------------------------------------------------

def kl_1d(n_e: int, L: float, n_modes: int):
    """Nystrom eigenpairs of exp(-|x - y| / L) on [0, 1].

    Trapezoid weights on the ``n_e + 1`` mesh nodes. Returns ``(mu, e)`` with
    ``mu`` descending and ``e[i]`` the i-th mode at the nodes, normalised in
    the discrete L2 norm (sum_j w_j e_j^2 = 1) and signed so that e(0) > 0.
    """
    x = np.linspace(0.0, 1.0, n_e + 1)
    w = np.full(n_e + 1, 1.0 / n_e)
    w[0] *= 0.5
    w[-1] *= 0.5
    C = np.exp(-np.abs(x[:, None] - x[None, :]) / L)
    sw = np.sqrt(w)
    B = sw[:, None] * C * sw[None, :]
    mu, V = np.linalg.eigh(B)
    order = np.argsort(mu)[::-1][:n_modes]
    mu = mu[order]
    E = (V[:, order] / sw[:, None]).T.copy()
    for i in range(E.shape[0]):
        if E[i, 0] < 0:
            E[i] = -E[i]
    return mu, E


def kl_2d(n_e: int, L: float, M: int):
    """Leading M eigenpairs of the separable 2D kernel exp(-|dx1|/L - |dx2|/L).

    Modes are products ``e_i(x1) e_j(x2)`` with ``lambda = mu_i mu_j``,
    sorted by lambda descending with ties broken by ``(i, j)`` ascending.
    Element values are products of the 1D element averages of the nodal
    modes. Returns ``(lam, phi, modes)`` with phi of shape (M, n_e, n_e).
    """
    if M == 0:
        return np.zeros(0), np.zeros((0, n_e, n_e)), []
    K1 = min(M + 1, n_e + 1)
    mu, E = kl_1d(n_e, L, K1)
    cand = []
    for i in range(K1):
        for j in range(K1):
            cand.append((-(mu[i] * mu[j]), i, j))
    cand.sort()
    modes = [(i, j) for (_, i, j) in cand[:M]]
    lam = np.array([mu[i] * mu[j] for (i, j) in modes])
    Ebar = 0.5 * (E[:, :-1] + E[:, 1:])  # element averages, (K1, n_e)
    phi = np.stack([np.outer(Ebar[j], Ebar[i]) for (i, j) in modes])  # [k, ey, ex]
    return lam, phi, modes


def node_coords(n_e: int):
    """Coordinates (x1, x2) of the interior nodes, x1 fastest."""
    t = np.arange(1, n_e) / n_e
    X1, X2 = np.meshgrid(t, t, indexing="xy")
    return X1.ravel(), X2.ravel()


def nodal_rhs(n_e: int, bump=None) -> np.ndarray:
    """f(x_i) at the interior nodes: f = 1, plus an optional Gaussian bump.

    ``bump = (A, w, c1, c2)`` adds ``A exp(-|x - c|^2 / (2 w^2))``.
    """
    x1, x2 = node_coords(n_e)
    f = np.ones_like(x1)
    if bump is not None:
        A, w, c1, c2 = bump
        f = f + A * np.exp(-((x1 - c1) ** 2 + (x2 - c2) ** 2) / (2.0 * w * w))
    return f


def qoi_weights(n_e: int, lo: float = 0.4, hi: float = 0.6):
    """Nodal weights of the subdomain quantity of interest over [lo, hi]^2.

    ``w_i = h^2`` for interior nodes inside the closed square, else 0.
    Returns ``(w_mean, w_var)`` with ``w_mean = w / sum(w)`` (subdomain mean
    of E[u]) and ``w_var = w`` (integral of Var[u]).
    """
    x1, x2 = node_coords(n_e)
    eps = 1e-12
    inside = (x1 >= lo - eps) & (x1 <= hi + eps) & (x2 >= lo - eps) & (x2 <= hi + eps)
    w = np.where(inside, 1.0 / (n_e * n_e), 0.0)
    return w / w.sum(), w


def make_problem(name, n_e, M, p, sigma, L, theta0=1.0, bump=None, family="hermite") -> Problem:
    lam, phi, modes = kl_2d(n_e, L, M)
    return Problem(
        name=name, n_e=n_e, M=M, p=p, theta0=float(theta0), sigma=float(sigma),
        L=float(L), s=np.sqrt(lam), phi=phi, f_nodal=nodal_rhs(n_e, bump), modes=modes,
        family=family,
    )


# The five workloads: small exact case, the 256^2 scale case (FP64 and FP32
# inner), the multi-problem batch, and the 512^2 differentiation case.
_NAMED = {
    "small": dict(n_e=16, M=4, p=2, sigma=0.2, L=0.5),
    "scale": dict(n_e=256, M=10, p=3, sigma=0.25, L=0.3),
    "grad": dict(n_e=512, M=8, p=3, sigma=0.2, L=0.4),
    "grad_small": dict(n_e=32, M=8, p=3, sigma=0.2, L=0.4),
    # the examples of Section 6: uniform variables with Legendre chaos on a
    # 10 x 10 mesh, mean 1, L = 0.5, CoV = sigma = 50 %, N = 4, degree 4
    "paper_legendre": dict(n_e=10, M=4, p=4, sigma=0.5, L=0.5, family="legendre"),
    # the 256^2 scale case with Legendre chaos
    "scale_legendre": dict(n_e=256, M=10, p=3, sigma=0.25, L=0.3, family="legendre"),
}


def named_problem(name: str, **override) -> Problem:
    cfg = dict(_NAMED[name])
    cfg.update(override)
    return make_problem(name, **cfg)


def batch_problems(seed: int = 0, count: int = 48, grids=(32, 64, 128, 256), max_P: int = 495):
    """Seeded set of independent SG problems of uneven size.

    Per problem: grid from ``grids``; then (M, p) with M in 4..10, p in 2..4,
    redrawn together until P <= max_P; then sigma ~ U[0.1, 0.3],
    L ~ U[0.2, 1.0] and a Gaussian bump (A ~ U[0.5, 2], w ~ U[0.05, 0.2],
    centre ~ U[0.2, 0.8]^2). sigma is redrawn while the coefficient margin is
    at most 0.05 (at most 100 draws, else ValueError).
    """
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        n_e = int(rng.choice(grids))
        while True:
            M = int(rng.integers(4, 11))
            p = int(rng.integers(2, 5))
            if n_chaos(M, p) <= max_P:
                break
        L = float(rng.uniform(0.2, 1.0))
        bump = (float(rng.uniform(0.5, 2.0)), float(rng.uniform(0.05, 0.2)),
                float(rng.uniform(0.2, 0.8)), float(rng.uniform(0.2, 0.8)))
        lam, phi, modes = kl_2d(n_e, L, M)
        for _ in range(100):
            sigma = float(rng.uniform(0.1, 0.3))
            prob = Problem(name=f"batch{b}", n_e=n_e, M=M, p=p, theta0=1.0, sigma=sigma, L=L,
                           s=np.sqrt(lam), phi=phi, f_nodal=nodal_rhs(n_e, bump), modes=modes)
            if prob.coefficient_margin() > 0.05:
                break
        else:
            raise ValueError(f"batch problem {b}: no sigma draw out of 100 keeps the coefficient margin above 0.05")
        out.append(prob)
    return out


def random_block(P: int, n: int, seed: int = 0) -> np.ndarray:
    """Seeded N(0, 1) block of shape (P, n)."""
    return np.random.default_rng(seed).standard_normal((P, n))
