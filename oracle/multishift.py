"""Multi-shift COCG for the shifted equations of one right-hand side.

TEST INFRASTRUCTURE (see the package header): only tests, the smoke check and
the benchmark's CPU leg use it.

The kernel convolutions of Section 3.1 (and the order-2 terms of Section 2)
solve (-L_h + kappa_r) u_r = f for several shifts kappa_r with the same f.
The Krylov spaces K_k(-L_h + kappa_r, f) do not depend on the shift, so one
COCG sequence of a seed system A = -L_h + kappa_s serves them all: with
sigma_r = kappa_r - kappa_s the residual of shift r after k steps is
collinear with the seed's, r_k^(r) = r_k / pi_k^(r), where pi_k^(r) is the
seed's residual polynomial evaluated at -sigma_r (the shifted COCG of
Takayama et al., Phys. Rev. B 73, 165108 (2006), after Frommer's shifted
BiCG).  All iterates start from zero.

The steps of one iteration k, in the order the method takes them:
  * direction of each shift: p^(r) = r_k / pi_k^(r) + beta_{k-1}^(r) p^(r),
    with beta_{k-1}^(r) = (pi_{k-1}^(r) / pi_k^(r))^2 beta_{k-1};
  * seed step: alpha_k = (r_k^T r_k) / (p^T A p) for the seed direction p
    (pi = 1 there), r_{k+1} = r_k - alpha_k A p;
  * shift polynomial: pi_{k+1}^(r) = (1 + alpha_k sigma_r) pi_k^(r)
    + (alpha_k beta_{k-1} / alpha_{k-1}) (pi_k^(r) - pi_{k-1}^(r));
  * shifted step: alpha_k^(r) = alpha_k pi_k^(r) / pi_{k+1}^(r),
    x^(r) += alpha_k^(r) p^(r);
  * beta_k = (r_{k+1}^T r_{k+1}) / (r_k^T r_k).
A shift whose residual |r_{k+1}| / |pi_{k+1}^(r)| has reached tol |f| is
frozen (its iterate and direction are no longer updated); the seed sequence
runs until every shift is frozen or maxit steps were taken.

Parity pins: every shift's result equals the spectral solve of its system to
the tolerance, and after any number of steps each shift's iterate equals the
textbook COCG iterate of its own system (the C oracle) after the same number
of steps.
"""
import numpy as np

from . import helmholtz


def solve(f: np.ndarray, kappas, h_xyz, N: int = 6, seed: int = 0, tol: float = 1e-10,
          maxit: int = 100000):
    """Returns (list of u_r, list of iterations per shift, seed steps taken).

    The iterations of shift r are the steps after which it was frozen (maxit
    if it never was)."""
    kap = [complex(k) for k in kappas]
    S = len(kap)
    f = np.asarray(f, dtype=np.complex128)
    sig = [k - kap[seed] for k in kap]
    x = [np.zeros_like(f) for _ in range(S)]
    p = [np.zeros_like(f) for _ in range(S)]
    r = f.copy()
    fn = np.linalg.norm(f)
    pi = [1.0 + 0j] * S
    pi_prev = [1.0 + 0j] * S
    running = [True] * S
    iters = [maxit] * S
    rho = complex(np.sum(r * r))
    alpha_prev, beta_prev = 1.0 + 0j, 0.0 + 0j
    k = 0
    if fn == 0.0:
        return x, [0] * S, 0
    while k < maxit and any(running):
        for j in range(S):
            if running[j] or j == seed:
                bj = (pi_prev[j] / pi[j]) ** 2 * beta_prev
                p[j] = r / pi[j] + bj * p[j]
        q = helmholtz.apply(p[seed], kap[seed], h_xyz, N)
        alpha = rho / complex(np.sum(p[seed] * q))
        r = r - alpha * q
        pi_next = [0j] * S
        for j in range(S):
            pi_next[j] = ((1.0 + alpha * sig[j]) * pi[j]
                          + (alpha * beta_prev / alpha_prev) * (pi[j] - pi_prev[j]))
            if running[j]:
                x[j] = x[j] + (alpha * pi[j] / pi_next[j]) * p[j]
        rho_new = complex(np.sum(r * r))
        beta = rho_new / rho
        rn = np.linalg.norm(r)
        k += 1
        for j in range(S):
            if running[j] and rn / abs(pi_next[j]) <= tol * fn:
                running[j] = False
                iters[j] = k
        pi_prev, pi = pi, pi_next
        alpha_prev, beta_prev, rho = alpha, beta, rho_new
    return x, iters, k
