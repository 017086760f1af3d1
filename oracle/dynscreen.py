"""FP64 oracle: dynamically screened ISTA / FISTA for the Lasso and the Group-Lasso.

TEST INFRASTRUCTURE ONLY (see the package docstring): never imported by the
product path.

Notation follows the paper: dictionary D (N x K) with atoms d_i, observation y,
penalty lambda, primal x, FISTA auxiliary u, dual variable theta, feasible dual
point v = mu * theta, sphere centre c and radius r, screened set I_t.

Readings of points the paper leaves open (each one is listed in the design doc):

* Step size: the paper sets L_t by the backtracking rule of Beck and Teboulle
  (Table 1) without constants.  step="constant" (the default) uses a constant
  L >= ||D||_2^2 supplied by the caller (default: the exact largest eigenvalue of
  D D^T); it stays valid after every screening because removing columns cannot
  increase the spectral norm.  step="backtracking" starts from L_0 (the caller's L,
  default the largest squared atom norm, or the largest ||D_g||_2^2 for groups)
  and, at every iteration, accepts the proximal point x' = prox(p - z / L) when
  ||D_t (x' - p)||^2 <= L ||x' - p||^2 -- for the quadratic data term this is exactly
  the condition F(x') <= Q_L(x', p) of that rule -- and otherwise multiplies L by
  eta (default 2) and repeats the iteration from the same p: such a rejected pass
  still produces its dual point, gap and screening radius (they do not depend on
  L), the FISTA sequence l_t does not advance, and the next pass evaluates theta at
  p restricted to the atoms that remain.  The solve stops only at an accepted step,
  so the returned x_t again has an objective no larger than the certified p.
* SpaRSA (rule="sparsa"): Table 1 gives it as ISTA whose L_t follows the
  Barzilai-Borwein rule of Wright, Nowak and Figueiredo, without its constants.
  Here, at iteration t with primal point p = x_{t-1} and proximal point x', the
  step d = x' - p is accepted when phi(x') <= max of the memory - (sigma / 2) L
  ||d||^2 (phi = P, the primal objective; sigma = bb_sigma, default 1e-5).  The
  memory holds phi at the current primal point and at the M = bb_memory iterates
  before it (default M = 0: monotone); its newest entry is refreshed when screening
  after a rejected step changed p.  phi(x') - phi(p) is formed as
  theta^T D d + ||D d||^2 / 2 + lambda (Omega(x') - Omega(p)), with the Omega
  difference summed term by term (|x'_i| - |p_i|, or for a group
  w_g d_g^T (x'_g + p_g) / (||x'_g|| + ||p_g||), the same difference of norms):
  that is the objective difference exactly, and its rounding error scales with d
  instead of with the objective, so the test keeps its meaning until the iterates
  stop moving (it is 0 for d = 0).  A rejected step is handled
  as in backtracking (L multiplied by eta, same p, the pass still screens and
  counts).  After an accepted step L becomes the Barzilai-Borwein value
  ||D_t d||^2 / ||d||^2 (kept when d = 0), clamped to [1e-30, 1e30]; the stopping
  iteration changes L in neither case.  d is the unscreened step (atoms removed by
  this iteration's test are cleared afterwards).  L_0 defaults as for backtracking.
* Initialisation X_0: x_0 = u_0 = 0 and l_0 = 1 by default; a caller's x0 gives
  x_0 = u_0 = x0 (the input X_0 of Algorithm 3).
* Dual scaling uses the correlations z_t = D_{t-1}^T theta_t of the current,
  already reduced dictionary, as the turnkey instance (Algorithm 5) does.
* Stopping: the paper's experiments stop after 200 iterations or when the objective's
  relative change falls below 1e-7; that rule is available (obj_tol, on the objective of
  the certified primal point of consecutive iterations).  By default the
  iteration stops when the duality gap between the primal point at which
  theta_t was evaluated (x_{t-1} for ISTA, u_{t-1} for FISTA) and the dual
  point v_t falls below gap_tol * ||y||^2, or after max_iter iterations.  The
  iterate returned is x_t, the proximal step taken from that primal point;
  with L >= ||D_t||^2 its objective is no larger, so the same gap bounds it.
  The last iteration does not screen, so the returned x_t is supported on the
  complement of the reported screened set.
* Tests on atoms that are not exactly unit-norm (storage rounding) use the
  general sphere bound of the group lemma with singleton groups: the margin of
  atom i is (1 - |d_i^T c|) / ||d_i||, and the DST3 centre is the projection of
  y/lambda onto the hyperplane {theta : d_*^T theta = 1}.  Both reduce to
  Lemmas 1 and 2 for unit atoms.
* Chambolle-Pock (rule="cp", Table 1): the dual iterate is carried from one iteration to
  the next, theta_t = (theta_{t-1} + sigma (D u_{t-1} - y)) / (1 + sigma), the primal step
  is x_t = prox(x_{t-1} - tau D^T theta_t, lambda tau), and u_t = x_t + phi (x_t - x_{t-1})
  with phi = 1/sqrt(1 + 2 gamma tau), tau <- phi tau, sigma <- sigma / phi.  The paper
  gives no gamma, tau_0 or sigma_0.  Reading: gamma = cp_gamma, default 0 (the basic
  method, constant steps, phi = 1); tau_0 = cp_tau, default 1/sqrt(L), and sigma_0 =
  cp_sigma, default 1/(tau_0 L), so tau sigma L = 1 with L >= ||D||_2^2 (the convergence
  condition); theta_0 = 0, x_0 = u_0 = 0.  Screening uses theta_t (dual scaling, Lemma 7).
  The gap certificate pairs theta_t's dual point with P(u_{t-1}) = ||D u_{t-1} - y||^2/2 +
  lambda Omega(u_{t-1}) (the residual the update already forms), and the solve returns
  u_{t-1}, the point so certified (x_t carries no such bound).  Screening removes atoms
  from x and u as for FISTA; theta, an N-vector, is untouched.
* Dynamic Dome test (the dome lemma of the section on dynamic tests): the region is the
  ball B(y/lambda, ||y/lambda - v_t||) cut by the half-space d_*^T theta <= 1.  The
  printed bounds Q^l, Q^u are those of that region for unit atoms except for their case
  split, which is written for the static dual point (theta = y, unit y: the split at
  t = -/+lambda_* with the constant lambda - 1 + lambda/lambda_*); for a general dual
  point the split falls where the ball's own maximiser leaves the half-space.  The
  region is used as stated, for atoms of any norm (dome_max, dome_margins), and the
  printed x^T d_i is read as y^T d_i.  Lasso only (the lemma is stated for the Lasso).
* Ties in the arg-max defining i_* / g_* go to the smallest index.  A radius
  whose square rounds below zero is clamped to zero.  An atom exactly at the
  threshold is kept (the test is a strict inequality).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class OracleResult:
    x: np.ndarray            # returned primal point (dense, length K)
    iters: int               # iterations run (0 in the trivial regime lambda >= lambda_*)
    converged: bool          # gap certificate reached gap_tol * ||y||^2
    lam: float
    lam_max: float
    gap: float               # P(p_{T-1}) - Dual(v_T): certificate of the last iteration
    primal_p: float          # P(p_{T-1}), p the point theta_T was evaluated at
    primal: float            # P(x_T), evaluated explicitly
    dual: float              # Dual(v_T)
    mu: float                # dual-scaling factor of the last iteration
    r_min: float             # smallest radius seen (inf when nothing was tested)
    screened: np.ndarray     # bool, length K: atoms in the reported screened set
    screened_groups: np.ndarray | None = None   # bool, length G (group problems)
    L: float = 0.0
    history: list = field(default_factory=list)


# ----------------------------------------------------------------------------
# Problem-level quantities
# ----------------------------------------------------------------------------

def lambda_max_lasso(D: np.ndarray, y: np.ndarray) -> tuple[float, int]:
    """lambda_* = ||D^T y||_inf and the first index attaining it.

    Section "Dynamic screening for the Lasso": for lambda >= lambda_* the
    solution is x = 0.  The signed atom d_* of Lemma 2 is sign(d_{i*}^T y) d_{i*}.
    """
    corr = np.abs(D.T @ y)
    i_star = int(np.argmax(corr))
    return float(corr[i_star]), i_star


def lambda_max_group(D: np.ndarray, y: np.ndarray, groups, w) -> tuple[float, int]:
    """Equation (gstar): g_* = argmax_g ||D_g^T y|| / w_g and lambda_* its value."""
    vals = np.array([np.linalg.norm(D[:, g].T @ y) / w[k] for k, g in enumerate(groups)])
    g_star = int(np.argmax(vals))
    return float(vals[g_star]), g_star


def spectral_norm_sq(D: np.ndarray) -> float:
    """||D||_2^2, the largest eigenvalue of D D^T (Lipschitz constant of the gradient)."""
    G = D @ D.T if D.shape[0] <= D.shape[1] else D.T @ D
    return float(np.linalg.eigvalsh(G)[-1])


def group_spectral_norms(D: np.ndarray, groups) -> np.ndarray:
    """||D_g||_2, the largest singular value of each sub-dictionary (Lemma 6)."""
    return np.array([np.linalg.norm(D[:, g], 2) if len(g) else 0.0 for g in groups])


# ----------------------------------------------------------------------------
# Proximal operators
# ----------------------------------------------------------------------------

def soft_threshold(v: np.ndarray, t: float) -> np.ndarray:
    """Equation (softTh): sign(v) * max(|v| - t, 0)."""
    return np.sign(v) * np.maximum(np.abs(v) - t, 0.0)


def group_soft_threshold(v: np.ndarray, t: float, groups, w) -> np.ndarray:
    """Equation (gr_softTh): v_g * max(0, (||v_g|| - t w_g) / ||v_g||), 0 when v_g = 0."""
    out = np.zeros_like(v)
    for k, g in enumerate(groups):
        nv = np.linalg.norm(v[g])
        if nv > 0.0:
            out[g] = max(0.0, (nv - t * w[k]) / nv) * v[g]
    return out


# ----------------------------------------------------------------------------
# Duality
# ----------------------------------------------------------------------------

def primal_objective(D, y, x, lam, omega) -> float:
    """Equation (1): 1/2 ||D x - y||^2 + lambda * Omega(x)."""
    res = D @ x - y
    return 0.5 * float(res @ res) + lam * omega


def dual_objective(v, y, lam) -> float:
    """Equations (dual) / (dual_glasso): 1/2 ||y||^2 - lambda^2/2 ||v - y/lambda||^2."""
    d = v - y / lam
    return 0.5 * float(y @ y) - 0.5 * lam * lam * float(d @ d)


def dual_scaling(theta: np.ndarray, y: np.ndarray, lam: float, s_bound: float) -> float:
    """Lemma 7 (and the mu of Lemmas 1-5): mu = [theta^T y / (lambda ||theta||^2)] clipped to [-s, s].

    s is 1/||D^T theta||_inf (Lasso) or min_g w_g / ||D_g^T theta|| (Group-Lasso);
    it is +inf when those correlations vanish.  theta = 0 gives mu = 0 (v = 0 is
    feasible).
    """
    nt2 = float(theta @ theta)
    if nt2 == 0.0:
        return 0.0
    return float(np.clip(float(theta @ y) / (lam * nt2), -s_bound, s_bound))


# ----------------------------------------------------------------------------
# Sphere centres and margins (Lemmas 1, 2, 4, 5, 6)
# ----------------------------------------------------------------------------

def lasso_center(D, y, lam, test, lam_max, i_star):
    """Centre c and rho^2 = ||y/lambda - c||^2 of the Lasso sphere tests.

    SAFE (Lemma 1): c = y/lambda, rho = 0, radius r = ||y/lambda - v||.
    DST3 (Lemma 2): c is the projection of y/lambda onto the hyperplane
    d_*^T theta = 1 bounding the half-space that contains the dual feasible set,
    r^2 = ||y/lambda - v||^2 - rho^2.  For a unit d_* this is
    c = y/lambda - (lambda_*/lambda - 1) d_*.
    """
    c0 = y / lam
    if test in ("none", "safe", "dome"):   # the dome's ball is SAFE's
        return c0, 0.0
    assert test == "dst3"
    d = D[:, i_star]
    d_star = d if float(d @ y) >= 0.0 else -d
    nd2 = float(d_star @ d_star)
    c = c0 - (float(d_star @ y) / lam - 1.0) * d_star / nd2
    e = c0 - c
    return c, float(e @ e)


def group_center(D, y, lam, test, groups, w, lam_max, g_star):
    """Centre c and rho^2 of the Group-Lasso sphere tests.

    GSAFE (Lemma 4): c = y/lambda.
    DGST3 (Lemma 5): n = D_{g*} D_{g*}^T y / lambda_*,
    c = (I - n n^T/||n||^2) y/lambda + n w_{g*}^2 / ||n||^2.
    """
    c0 = y / lam
    if test in ("none", "gsafe"):
        return c0, 0.0
    assert test == "dgst3"
    Dg = D[:, groups[g_star]]
    n = Dg @ (Dg.T @ y) / lam_max
    nn = float(n @ n)
    c = c0 - n * float(n @ c0) / nn + n * (w[g_star] ** 2) / nn
    e = c0 - c
    return c, float(e @ e)


def lasso_margins(D, c, test):
    """Per-atom margin m_i = (1 - |d_i^T c|) / ||d_i||: atom i is screened when m_i > r.

    Lemmas 1-2 for unit atoms; Lemma 6 with singleton groups otherwise.  A zero
    atom has margin +inf; with no test every margin is -inf.
    """
    K = D.shape[1]
    if test == "none":
        return np.full(K, -np.inf)
    nu = np.linalg.norm(D, axis=0)
    corr = np.abs(D.T @ c)
    m = np.full(K, np.inf)
    nz = nu > 0
    m[nz] = (1.0 - corr[nz]) / nu[nz]
    return m


def dome_max(U, c, R, n, h, points=False):
    """Largest u^T theta over the dome {||theta - c|| <= R} cut by {n^T theta <= h} (n a
    unit vector, R at least the distance n^T c - h from c to the plane, so the dome is not
    empty), for each column u of U (R a scalar or one radius per column).  If the ball's
    own maximiser c + R u/||u|| lies in the half-space it is the answer; otherwise the
    maximum is taken on the cutting plane, over the disc of centre c' = c - (n^T c - h) n
    and radius sqrt(R^2 - (n^T c - h)^2), at c' plus that radius times the unit component
    of u orthogonal to n.  With points=True the maximising points are returned too."""
    U = np.asarray(U, dtype=np.float64)
    U = U[:, None] if U.ndim == 1 else U
    R = np.broadcast_to(np.asarray(R, dtype=np.float64), (U.shape[1],))
    nu = np.linalg.norm(U, axis=0)
    uc = U.T @ c
    un = U.T @ n
    delta = float(n @ c) - h
    in_half = float(n @ c) + R * un / nu <= h      # n^T (c + R u/||u||) <= h
    r2 = np.sqrt(np.maximum(R * R - delta * delta, 0.0))
    npn = np.sqrt(np.maximum(nu * nu - un * un, 0.0))   # ||u - (u^T n) n||
    val = np.where(in_half, uc + R * nu, uc - delta * un + r2 * npn)
    if not points:
        return val
    up = U - np.outer(n, un)
    t_ball = c[:, None] + U * (R / nu)
    t_disc = (c - delta * n)[:, None] + up * (r2 / np.where(npn > 0, npn, 1.0))
    return val, np.where(in_half, t_ball, t_disc)


def dome_setup(D, y, lam, i_star):
    """The dome of the dynamic Dome test (Lemma 'dynamic dome'): centre y/lambda, and the
    half-space d_*^T theta <= 1 of the atom attaining lambda_* (signed so that
    d_*^T y = lambda_*), as a unit normal n and offset h = 1/||d_*||."""
    d = D[:, i_star]
    d_star = d if float(d @ y) >= 0.0 else -d
    nd = float(np.linalg.norm(d_star))
    return y / lam, d_star / nd, 1.0 / nd


def dome_margins(D, y, lam, i_star, iters=200):
    """Per-atom threshold of the dynamic Dome test: the largest R for which the maximum of
    |d_i^T theta| over the dome B(y/lambda, R) cut by d_*^T theta <= 1 stays below 1.  That
    maximum grows with R, so atom i is screened at radius R_t = ||y/lambda - v_t|| exactly
    when R_t < m_i.  Found by bisection on that definition (both signs of d_i), starting
    from the smallest radius with a non-empty dome, delta = the distance from y/lambda to
    the plane: an atom whose bound stays below 1 at every radius has m_i = +inf, one that
    reaches 1 already at delta has m_i = delta (never screened, since R_t >= delta), as
    has d_* itself."""
    c, n, h = dome_setup(D, y, lam, i_star)
    delta = float(n @ c) - h
    K = D.shape[1]

    def f(R):
        return np.maximum(dome_max(D, c, R, n, h), dome_max(-D, c, R, n, h))

    big = (delta + 1.0) * 1e12
    never = f(np.full(K, delta)) >= 1.0
    always = f(np.full(K, big)) < 1.0
    lo = np.full(K, delta)
    hi = np.full(K, big)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        below = f(mid) < 1.0
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    m = lo
    m[never] = delta
    m[always] = np.inf
    # d_* itself attains d_*^T theta = 1 on the cutting plane at every radius (its bound is
    # exactly 1, which rounding can put on either side): it is never screened
    m[i_star] = delta
    return m


def group_margins(D, c, test, groups, w, gnorm):
    """Per-group margin m_g = (w_g - ||D_g^T c||) / ||D_g||_2 (Lemmas 4, 5 and 6)."""
    G = len(groups)
    if test == "none":
        return np.full(G, -np.inf)
    m = np.full(G, np.inf)
    for k, g in enumerate(groups):
        if gnorm[k] > 0:
            m[k] = (w[k] - np.linalg.norm(D[:, g].T @ c)) / gnorm[k]
    return m


# ----------------------------------------------------------------------------
# Algorithm 3 instantiated with ISTA / FISTA (Table 1)
# ----------------------------------------------------------------------------

def _radius(R2, rho2, test):
    if test == "none":
        return np.inf
    if test in ("safe", "gsafe", "dome"):
        return float(np.sqrt(R2))
    return float(np.sqrt(max(R2 - rho2, 0.0)))


def _trivial(K, lam, lam_max, L, G=None):
    return OracleResult(
        x=np.zeros(K), iters=0, converged=True, lam=lam, lam_max=lam_max, gap=0.0,
        primal_p=0.0, primal=0.0, dual=0.0, mu=0.0, r_min=0.0,
        screened=np.ones(K, dtype=bool),
        screened_groups=None if G is None else np.ones(G, dtype=bool), L=L)


def _bb_step(Dd, d, L):
    """Barzilai-Borwein step of SpaRSA after an accepted step d: ||D d||^2 / ||d||^2 (the
    Rayleigh quotient of D^T D along d), clamped to [1e-30, 1e30]; L is kept when d = 0."""
    dd = float(d @ d)
    if not dd > 0.0:
        return L
    return float(min(max(float(Dd @ Dd) / dd, 1e-30), 1e30))


def solve_lasso(D, y, *, lam=None, lam_ratio=None, rule="fista", test="dst3", L=None,
                max_iter=1000, gap_tol=1e-6, record=False, screening="dynamic",
                step="constant", eta=2.0, bb_memory=0, bb_sigma=1e-5, cp_tau=None,
                cp_sigma=None, cp_gamma=0.0, x0=None, obj_tol=0.0) -> OracleResult:
    """Lasso (equation (lasso)) by Algorithm 3 with the ISTA or FISTA update of Table 1.

    x0: the initial point X_0 of Algorithm 3 (default 0): x_0 = u_0 = x0, l_0 = 1 (the
    Chambolle-Pock dual iterate still starts at 0).
    obj_tol > 0 adds the stopping rule of the experiments section: stop once the objective
    of the certified primal point changes by at most obj_tol relative between two
    consecutive accepted iterations whose primal points are both non-zero.

    Each iteration: the update (theta_t = D_{t-1} p - y, z_t = D_{t-1}^T theta_t,
    x_t = prox(p - z_t / L, lambda / L), FISTA momentum), the dual point
    v_t = mu_t theta_t, the sphere radius r_t of the chosen test (SAFE Lemma 1,
    DST3 Lemma 2, the dynamic Dome test with the SAFE radius and the thresholds of
    dome_margins, or none), the screened set I_t = {i : m_i > r_t} U I_{t-1}, and the
    reduction of D and of the primal variables to the complement of I_t.

    screening="static" runs the test once, at the first iteration, where the dual point
    from x_0 = 0 makes it the static test of Algorithms 1 and 4 (static SAFE, ST3); the
    first update does not depend on the atoms that test removes (their prox output is 0).
    step="backtracking" sets L_t by the backtracking rule (module docstring); L is then L_0.
    rule="sparsa" is ISTA with the Barzilai-Borwein step and its acceptance test (module
    docstring; bb_memory, bb_sigma, eta); L is then L_0.  rule="cp" is Chambolle-Pock
    (module docstring; cp_tau, cp_sigma, cp_gamma; L >= ||D||_2^2 sets the default steps).
    """
    D = np.asarray(D, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    N, K = D.shape
    assert test in ("none", "safe", "dst3", "dome") and rule in ("ista", "fista", "sparsa", "cp")
    assert rule != "cp" or (step == "constant" and cp_gamma >= 0.0)
    assert step in ("constant", "backtracking") and eta > 1.0
    assert rule != "sparsa" or (step == "constant" and bb_memory >= 0 and bb_sigma >= 0.0)
    lam_max, i_star = lambda_max_lasso(D, y)
    if lam is None:
        lam = float(lam_ratio) * lam_max
    if L is None:
        L = spectral_norm_sq(D) if step == "constant" and rule != "sparsa" \
            else float(np.max(np.sum(D * D, axis=0)))
    if lam >= lam_max:
        return _trivial(K, lam, lam_max, L)

    c, rho2 = lasso_center(D, y, lam, test, lam_max, i_star)
    m = dome_margins(D, y, lam, i_star) if test == "dome" else lasso_margins(D, c, test)
    yy = float(y @ y)

    screened = np.zeros(K, dtype=bool)          # I_0 = empty set
    active = np.arange(K)                       # complement of I_0
    Dt = D                                      # D_0 = D
    x = np.zeros(K) if x0 is None else np.array(x0, dtype=np.float64)   # x_0
    u = x.copy()                                # u_0
    l_prev = 1.0                                # l_0
    r_min = np.inf
    hist = []
    phis, new_point = [], True                  # SpaRSA: phi at the last M + 1 iterates
    if rule == "cp":                            # Chambolle-Pock steps and dual iterate
        tau = float(cp_tau) if cp_tau else 1.0 / np.sqrt(L)
        sigma = float(cp_sigma) if cp_sigma else 1.0 / (tau * L)
        theta_cp = np.zeros(N)
    converged = False
    primal_prev, prev_accepted, omega_prev = 0.0, True, 0.0   # the objective-change rule
    for t in range(1, max_iter + 1):
        # ---- optimisation update (Table 1) ----
        p = u if rule in ("fista", "cp") else x
        omega_p = float(np.abs(p).sum())
        if rule == "cp":
            res = Dt @ p - y
            theta = (theta_cp + sigma * res) / (1.0 + sigma)
            z = Dt.T @ theta
            x_new = soft_threshold(x - tau * z, lam * tau)
            phi = 1.0 / np.sqrt(1.0 + 2.0 * cp_gamma * tau)
            primal_p = 0.5 * float(res @ res) + lam * omega_p
        else:
            theta = Dt @ p - y
            z = Dt.T @ theta
            x_new = soft_threshold(p - z / L, lam / L)
            primal_p = 0.5 * float(theta @ theta) + lam * omega_p
        accepted = True
        if step == "backtracking":  # F(x_new) <= Q_L(x_new, p)  <=>  ||D d||^2 <= L ||d||^2
            d = x_new - p
            Dd = Dt @ d
            accepted = float(Dd @ Dd) <= L * float(d @ d)
        elif rule == "sparsa":      # sufficient decrease against the memory
            if new_point:
                phis = (phis + [primal_p])[-(bb_memory + 1):]
            else:
                phis[-1] = primal_p
            d = x_new - p
            Dd = Dt @ d
            dphi = float(theta @ Dd) + 0.5 * float(Dd @ Dd) \
                + lam * float(np.sum(np.abs(x_new) - np.abs(p)))
            phi_new = primal_p + dphi
            accepted = dphi + (primal_p - max(phis)) <= -0.5 * bb_sigma * L * float(d @ d)
        if rule == "fista":
            l_new = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * l_prev * l_prev))
            u_new = x_new + ((l_prev - 1.0) / l_new) * (x_new - x)
        elif rule == "cp":
            l_new = l_prev
            u_new = x_new + phi * (x_new - x)
        else:
            l_new = l_prev
            u_new = x_new
        # ---- dual point by dual scaling (Lemma 1 / Algorithm 5) ----
        zinf = float(np.max(np.abs(z))) if z.size else 0.0
        s_bound = 1.0 / zinf if zinf > 0.0 else np.inf
        mu = dual_scaling(theta, y, lam, s_bound)
        v = mu * theta
        # ---- duality-gap certificate of p ----
        dual = dual_objective(v, y, lam)
        gap = primal_p - dual
        dv = y / lam - v
        r = _radius(float(dv @ dv), rho2, test)
        r_min = min(r_min, r)
        if record:
            hist.append(dict(t=t, n_active=int(active.size), nnz=int(np.count_nonzero(x_new)),
                             nnz_p=int(np.count_nonzero(p)), r=r, gap=gap, mu=mu, L=L,
                             accepted=accepted, primal_p=primal_p))
            if step == "backtracking" or rule == "sparsa":  # candidate, primal point, active set
                hist[-1].update(cand=x_new.copy(), p=p.copy(), active=active.copy())
            if rule == "sparsa":
                hist[-1].update(phi_new=phi_new, phi_ref=max(phis))
            if rule == "cp":
                hist[-1].update(theta=theta.copy(), tau=tau, sigma=sigma, x_prev=x.copy())
        obj_stop = (obj_tol > 0.0 and accepted and prev_accepted and t > 1
                    and omega_p > 0.0 and omega_prev > 0.0
                    and abs(primal_prev - primal_p) <= obj_tol * primal_p)
        primal_prev, prev_accepted, omega_prev = primal_p, accepted, omega_p
        converged = (gap_tol > 0.0 and gap <= gap_tol * yy and accepted) or obj_stop
        if not accepted:
            # rejected step: keep p, grow L; at the iteration limit return the last accepted x
            x_new, u_new, l_new = x, u, l_prev
            if t < max_iter:
                L *= eta
        elif rule == "sparsa" and not converged and t < max_iter:
            L = _bb_step(Dd, d, L)
        new_point = accepted
        if rule == "cp":
            if converged or t == max_iter:
                x_new = p.copy()        # the point the certificate is about
            else:
                theta_cp, tau, sigma = theta, tau * phi, sigma / phi
        if converged or t == max_iter:
            break
        # ---- screening: I_t = {i : T_v(i)} U I_{t-1}, then reduce D and X ----
        if screening == "dynamic" or t == 1:
            screened = screened | (m > r)
        keep = ~screened[active]
        if not keep.all():
            Dt = Dt[:, keep]
            active = active[keep]
            x_new = x_new[keep]
            u_new = u_new[keep]
        x, u, l_prev = x_new, u_new, l_new

    x_full = np.zeros(K)
    x_full[active] = x_new
    primal = primal_objective(D, y, x_full, lam, float(np.abs(x_full).sum()))
    return OracleResult(x=x_full, iters=t, converged=converged, lam=lam, lam_max=lam_max,
                        gap=gap, primal_p=primal_p, primal=primal, dual=dual, mu=mu,
                        r_min=r_min, screened=screened, L=L, history=hist)


def _as_groups(K, groups):
    """Accept either a list of index arrays (any partition) or CSR offsets of contiguous groups."""
    if isinstance(groups, np.ndarray) and groups.ndim == 1 and groups.dtype.kind in "iu" \
            and groups.size >= 2 and groups[0] == 0 and groups[-1] == K:
        return [np.arange(groups[k], groups[k + 1]) for k in range(groups.size - 1)]
    return [np.asarray(g, dtype=np.int64) for g in groups]


def solve_group_lasso(D, y, groups, w=None, *, lam=None, lam_ratio=None, rule="ista",
                      test="dgst3", L=None, max_iter=1000, gap_tol=1e-6,
                      record=False, screening="dynamic", step="constant",
                      eta=2.0, bb_memory=0, bb_sigma=1e-5, cp_tau=None, cp_sigma=None,
                      cp_gamma=0.0, x0=None, obj_tol=0.0) -> OracleResult:
    """Group-Lasso (equation (group-lasso)) by Algorithm 3 with ISTA / FISTA.

    x0: the initial point X_0 (default 0) and obj_tol, as in solve_lasso.

    groups: a partition of range(K) (list of index arrays, or contiguous CSR
    offsets); w: group weights, default sqrt(|g|).  Tests: GSAFE (Lemma 4),
    DGST3 (Lemma 5) or none; the screening unit is the group.  screening="static"
    runs the test once, at the first iteration (the static group tests).  step as in
    solve_lasso (the default L_0 for backtracking and SpaRSA is max_g ||D_g||_2^2);
    rule="sparsa" as in solve_lasso, with phi the Group-Lasso objective; rule="cp" as in
    solve_lasso, with the group shrinkage as the prox.
    """
    D = np.asarray(D, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    N, K = D.shape
    groups = _as_groups(K, groups)
    G = len(groups)
    w = np.sqrt([len(g) for g in groups]).astype(np.float64) if w is None else np.asarray(w, np.float64)
    assert test in ("none", "gsafe", "dgst3") and rule in ("ista", "fista", "sparsa", "cp")
    assert rule != "cp" or (step == "constant" and cp_gamma >= 0.0)
    assert screening in ("dynamic", "static")
    assert step in ("constant", "backtracking") and eta > 1.0
    assert rule != "sparsa" or (step == "constant" and bb_memory >= 0 and bb_sigma >= 0.0)
    lam_max, g_star = lambda_max_group(D, y, groups, w)
    if lam is None:
        lam = float(lam_ratio) * lam_max
    gnorm = group_spectral_norms(D, groups)
    if L is None:
        L = spectral_norm_sq(D) if step == "constant" and rule != "sparsa" \
            else float(np.max(gnorm) ** 2)
    if lam >= lam_max:
        return _trivial(K, lam, lam_max, L, G)

    c, rho2 = group_center(D, y, lam, test, groups, w, lam_max, g_star)
    m = group_margins(D, c, test, groups, w, gnorm)
    yy = float(y @ y)

    screened_g = np.zeros(G, dtype=bool)
    act_g = np.arange(G)

    def layout(ag):
        cols = np.concatenate([groups[k] for k in ag]) if len(ag) else np.zeros(0, np.int64)
        local, pos = [], 0
        for k in ag:
            local.append(np.arange(pos, pos + len(groups[k])))
            pos += len(groups[k])
        return cols, local

    cols, local = layout(act_g)
    Dt = D[:, cols]
    x = np.zeros(cols.size) if x0 is None else np.asarray(x0, dtype=np.float64)[cols]
    u = x.copy()
    l_prev = 1.0
    r_min = np.inf
    hist = []
    phis, new_point = [], True
    if rule == "cp":
        tau = float(cp_tau) if cp_tau else 1.0 / np.sqrt(L)
        sigma = float(cp_sigma) if cp_sigma else 1.0 / (tau * L)
        theta_cp = np.zeros(N)
    converged = False
    primal_prev, prev_accepted, omega_prev = 0.0, True, 0.0   # the objective-change rule
    for t in range(1, max_iter + 1):
        wa = w[act_g]
        p = u if rule in ("fista", "cp") else x
        omega_p = float(sum(wa[j] * np.linalg.norm(p[lg]) for j, lg in enumerate(local)))
        if rule == "cp":
            res = Dt @ p - y
            theta = (theta_cp + sigma * res) / (1.0 + sigma)
            z = Dt.T @ theta
            x_new = group_soft_threshold(x - tau * z, lam * tau, local, wa)
            phi = 1.0 / np.sqrt(1.0 + 2.0 * cp_gamma * tau)
            primal_p = 0.5 * float(res @ res) + lam * omega_p
        else:
            theta = Dt @ p - y
            z = Dt.T @ theta
            x_new = group_soft_threshold(p - z / L, lam / L, local, wa)
            primal_p = 0.5 * float(theta @ theta) + lam * omega_p
        accepted = True
        if step == "backtracking":  # F(x_new) <= Q_L(x_new, p)  <=>  ||D d||^2 <= L ||d||^2
            d = x_new - p
            Dd = Dt @ d
            accepted = float(Dd @ Dd) <= L * float(d @ d)
        elif rule == "sparsa":
            if new_point:
                phis = (phis + [primal_p])[-(bb_memory + 1):]
            else:
                phis[-1] = primal_p
            d = x_new - p
            Dd = Dt @ d
            domega = 0.0            # Omega(x') - Omega(p), group by group
            for j, lg in enumerate(local):
                den = np.linalg.norm(x_new[lg]) + np.linalg.norm(p[lg])
                if den > 0.0:       # ||a|| - ||b|| = (a - b)^T (a + b) / (||a|| + ||b||)
                    domega += wa[j] * float(d[lg] @ (x_new[lg] + p[lg])) / den
            dphi = float(theta @ Dd) + 0.5 * float(Dd @ Dd) + lam * domega
            phi_new = primal_p + dphi
            accepted = dphi + (primal_p - max(phis)) <= -0.5 * bb_sigma * L * float(d @ d)
        if rule == "fista":
            l_new = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * l_prev * l_prev))
            u_new = x_new + ((l_prev - 1.0) / l_new) * (x_new - x)
        elif rule == "cp":
            l_new = l_prev
            u_new = x_new + phi * (x_new - x)
        else:
            l_new = l_prev
            u_new = x_new
        zg = np.array([np.linalg.norm(z[lg]) for lg in local])
        pos = zg > 0.0
        s_bound = float(np.min(wa[pos] / zg[pos])) if pos.any() else np.inf
        mu = dual_scaling(theta, y, lam, s_bound)
        v = mu * theta
        dual = dual_objective(v, y, lam)
        gap = primal_p - dual
        dv = y / lam - v
        r = _radius(float(dv @ dv), rho2, {"gsafe": "safe", "dgst3": "dst3"}.get(test, test))
        r_min = min(r_min, r)
        if record:
            hist.append(dict(t=t, n_active=int(cols.size), n_active_groups=int(act_g.size),
                             nnz=int(np.count_nonzero(x_new)), nnz_p=int(np.count_nonzero(p)),
                             r=r, gap=gap, mu=mu, L=L, accepted=accepted, primal_p=primal_p))
            if rule == "sparsa":
                hist[-1].update(phi_new=phi_new, phi_ref=max(phis))
            if rule == "cp":
                hist[-1].update(theta=theta.copy(), tau=tau, sigma=sigma, x_prev=x.copy())
        obj_stop = (obj_tol > 0.0 and accepted and prev_accepted and t > 1
                    and omega_p > 0.0 and omega_prev > 0.0
                    and abs(primal_prev - primal_p) <= obj_tol * primal_p)
        primal_prev, prev_accepted, omega_prev = primal_p, accepted, omega_p
        converged = (gap_tol > 0.0 and gap <= gap_tol * yy and accepted) or obj_stop
        if not accepted:
            x_new, u_new, l_new = x, u, l_prev
            if t < max_iter:
                L *= eta
        elif rule == "sparsa" and not converged and t < max_iter:
            L = _bb_step(Dd, d, L)
        new_point = accepted
        if rule == "cp":
            if converged or t == max_iter:
                x_new = p.copy()
            else:
                theta_cp, tau, sigma = theta, tau * phi, sigma / phi
        if converged or t == max_iter:
            break
        if screening == "dynamic" or t == 1:
            screened_g = screened_g | (m > r)
        keep_g = ~screened_g[act_g]
        if not keep_g.all():
            keep_cols = np.concatenate([local[j] for j in range(act_g.size) if keep_g[j]]) \
                if keep_g.any() else np.zeros(0, np.int64)
            act_g = act_g[keep_g]
            cols, local = layout(act_g)
            Dt = D[:, cols]
            x_new = x_new[keep_cols]
            u_new = u_new[keep_cols]
        x, u, l_prev = x_new, u_new, l_new

    x_full = np.zeros(K)
    x_full[cols] = x_new
    omega = float(sum(w[k] * np.linalg.norm(x_full[g]) for k, g in enumerate(groups)))
    primal = primal_objective(D, y, x_full, lam, omega)
    screened = np.zeros(K, dtype=bool)
    for k in np.flatnonzero(screened_g):
        screened[groups[k]] = True
    return OracleResult(x=x_full, iters=t, converged=converged, lam=lam, lam_max=lam_max,
                        gap=gap, primal_p=primal_p, primal=primal, dual=dual, mu=mu,
                        r_min=r_min, screened=screened, screened_groups=screened_g, L=L,
                        history=hist)


# ----------------------------------------------------------------------------
# Certified inactive sets (for safety checks) and the flops model
# ----------------------------------------------------------------------------

def certified_inactive_lasso(D, y, lam, x):
    """Atoms provably zero at the exact Lasso solution, from a near-optimal x.

    v = mu (D x - y) with mu by dual scaling over the full D is dual feasible;
    the dual objective is lambda^2-strongly concave, so ||theta_opt - v|| <=
    sqrt(2 gap)/lambda, and |d_i^T v| + ||d_i|| sqrt(2 gap)/lambda < 1 implies
    |d_i^T theta_opt| < 1, hence x_opt_i = 0 by the optimality conditions
    (equation (primaldual)).  Returns (mask, gap).
    """
    theta = D @ x - y
    zinf = float(np.max(np.abs(D.T @ theta)))
    mu = dual_scaling(theta, y, lam, 1.0 / zinf if zinf > 0 else np.inf)
    v = mu * theta
    gap = primal_objective(D, y, x, lam, float(np.abs(x).sum())) - dual_objective(v, y, lam)
    rad = np.sqrt(2.0 * max(gap, 0.0)) / lam
    nu = np.linalg.norm(D, axis=0)
    return np.abs(D.T @ v) + nu * rad < 1.0, gap


def certified_inactive_group(D, y, lam, x, groups, w=None):
    """Group version (equation (primaldualKKT_glasso)); returns (atom mask, group mask, gap)."""
    N, K = D.shape
    groups = _as_groups(K, groups)
    w = np.sqrt([len(g) for g in groups]) if w is None else np.asarray(w, np.float64)
    theta = D @ x - y
    zg = np.array([np.linalg.norm(D[:, g].T @ theta) for g in groups])
    pos = zg > 0
    mu = dual_scaling(theta, y, lam, float(np.min(w[pos] / zg[pos])) if pos.any() else np.inf)
    v = mu * theta
    omega = float(sum(w[k] * np.linalg.norm(x[g]) for k, g in enumerate(groups)))
    gap = primal_objective(D, y, x, lam, omega) - dual_objective(v, y, lam)
    rad = np.sqrt(2.0 * max(gap, 0.0)) / lam
    gnorm = group_spectral_norms(D, groups)
    gmask = np.array([np.linalg.norm(D[:, g].T @ v) + gnorm[k] * rad < w[k]
                      for k, g in enumerate(groups)])
    amask = np.zeros(K, dtype=bool)
    for k in np.flatnonzero(gmask):
        amask[groups[k]] = True
    return amask, gmask, gap


def flops_none(history, N, K, n_groups=None):
    """Flops model of the experiments section without screening (flops_N).

    Lasso: sum_t [(K + ||x_t||_0) N + 4 K + N];
    Group-Lasso: sum_t [(K + ||x_t||_0) N + 4 K + N + 3 |G|].
    """
    tot = 0
    for h in history:
        tot += (K + h["nnz"]) * N + 4 * K + N + (0 if n_groups is None else 3 * n_groups)
    return tot


def flops_static(history, N, K, n_kept, n_groups=None):
    """Flops model of the experiments section for static screening (flops_S): K N for the
    test, then every iteration on the |I^c_0| = n_kept atoms the test kept.

    Lasso: K N + sum_t [(|I^c_0| + ||x_t||_0) N + 4 |I^c_0| + N];
    Group-Lasso: the same plus 3 |G| per iteration.
    """
    tot = K * N
    for h in history:
        tot += (n_kept + h["nnz"]) * N + 4 * n_kept + N + (0 if n_groups is None else 3 * n_groups)
    return tot


def flops_dynamic(history, N, n_groups=None):
    """Flops model of the experiments section for the dynamic strategy.

    Lasso: sum_t [(|I^c_t| + ||x_t||_0) N + 6 |I^c_t| + 5 N];
    Group-Lasso: sum_t [(|I^c_t| + ||x_t||_0) N + 7 |I^c_t| + 5 N + 5 |G|].
    """
    tot = 0
    for h in history:
        a, s = h["n_active"], h["nnz"]
        if n_groups is None:
            tot += (a + s) * N + 6 * a + 5 * N
        else:
            tot += (a + s) * N + 7 * a + 5 * N + 5 * n_groups
    return tot
