"""The refinement-free Calderon multiplicative preconditioner (RF-CMP).

Follows Sec. 2 (projectors), Sec. 3 (eq. NewFormulation, outer matrix P_o,
middle matrix P_m, recovery j = P_o i), Sec. 3.4 (adjoint by conjugation, CG and
its iteration bound) and Sec. 4 (implemented scalings alpha, beta, gamma
estimated by power iteration).  All matrices are dense float64/complex128.

Notation: Sig = Sigma (star matrix), Lam = Lambda (loop matrix),
L = Sig^T Sig, Lp = L^+ (Moore-Penrose), G_ll, G_pp = diag(1/A), G_tp.

  P_S   = Sig Lp Sig^T,             P_LH = I - P_S
  P_gS  = Sig Lp G_tp^-1 Sig^T                              (Sec. 3)
  P_o   = P_LH/alpha + i P_s/beta,  P_s in {P_S (Sec. 4), P_gS (Sec. 3)}
  P_mL  = Lam G_ll^-1 Lam^T/alpha^2 + P_LH/gamma
  P_mS  = Sig Lp G_pp^-1 Lp Sig^T/beta^2
  A     = P_o^H T^H (P_mL + P_mS) T P_o,   b = -P_o^H T^H P_m e,   j = P_o i
  T     = i k T_A + Sig V Sig^T/(i k)
"""

import numpy as np

from . import grams

__all__ = ["Preconditioner", "cg", "power_norm", "iteration_bound", "efie_condition"]


class Preconditioner:
    """Dense RF-CMP operators for one mesh, one wavenumber and one (T_A, V)."""

    def __init__(self, top, TA, V, k, outer_star="sigma"):
        if outer_star not in ("sigma", "gsigma"):
            raise ValueError("outer_star must be 'sigma' or 'gsigma'")
        self.top, self.TA, self.V, self.k = top, TA, V, float(k)
        self.outer_star = outer_star
        Sig, Lam = top.Sigma, top.Lambda
        C = top.C
        L = grams.laplacian(top)
        J = np.full((C, C), 1.0 / C)
        # Sec. 3.2: (Sig^T Sig + 1 1^T/C)^-1 = (Sig^T Sig)^+ + 1 1^T/C
        self.Lp = np.linalg.inv(L + J) - J
        self.P_S = Sig @ self.Lp @ Sig.T
        self.P_LH = np.eye(top.N) - self.P_S
        self.Gll_inv = np.linalg.inv(grams.gram_ll(top))
        self.Gtp = grams.gram_tp(top)
        self.Gtp_inv = np.linalg.inv(self.Gtp)
        self.P_gS = Sig @ self.Lp @ self.Gtp_inv @ Sig.T
        self.P_s = self.P_S if outer_star == "sigma" else self.P_gS
        self.Gpp_inv = np.linalg.inv(grams.gram_pp(top))
        self.MS_hat = Sig @ self.Lp @ self.Gpp_inv @ self.Lp @ Sig.T   # P_mS without 1/beta^2
        self.ML_hat = Lam @ self.Gll_inv @ Lam.T
        self.TPhi = Sig @ V @ Sig.T
        self.alpha = self.beta = self.gamma = None

    # ----- scalings (Sec. 4) -----------------------------------------------
    def set_scalings(self, alpha, beta, gamma):
        self.alpha, self.beta, self.gamma = float(alpha), float(beta), float(gamma)

    def k_scalings(self):
        """alpha = sqrt(k), beta = 1/sqrt(k), gamma = k reproduce Sec. 3."""
        k = self.k
        self.set_scalings(np.sqrt(k), 1.0 / np.sqrt(k), k)

    def scaling_operators(self):
        """The three HPD operators whose 2-norms define alpha, beta, gamma.

        In the norms the two potential blocks are read as the two summands of
        the EFIE matrix, i k T_A and T_Phi/(i k); the k factors are applied in
        ``power_scalings``.  The unscaled star middle matrix is used inside
        beta's norm.
        """
        TA, P_LH, P_S = self.TA, self.P_LH, self.P_S
        TAc = np.conj(TA)
        Oa = lambda v: P_LH @ (TAc @ (self.ML_hat @ (TA @ (P_LH @ v))))
        Og = lambda v: P_LH @ (TAc @ (P_LH @ (TA @ (P_LH @ v))))
        Ob = lambda v: P_S @ (np.conj(self.TPhi) @ (self.MS_hat @ (self.TPhi @ (P_S @ v))))
        return Oa, Ob, Og

    def power_scalings(self, start, steps=30, tol=0.0):
        """alpha, beta, gamma (Sec. 4) from power iterations from ``start``.

        The three operators are iterated side by side.  With tol = 0 all
        ``steps`` steps run.  With tol > 0 the scalings are formed every
        POWER_CHECK steps, and the iteration stops at the first check from
        2 POWER_CHECK steps on where each of alpha, beta, gamma moved by less
        than tol (relative) since the previous check; ``steps`` is then the
        most it runs.  Returns (alpha, beta, gamma, (la, lb, lg), steps run)."""
        k = self.k
        ops = self.scaling_operators()
        v = [start / np.linalg.norm(start) for _ in range(3)]
        lam = [0.0, 0.0, 0.0]

        def scal(la, lb, lg):
            alpha = (k * k * la) ** 0.25
            return alpha, (lb / (k * k)) ** 0.25, k * k * lg / alpha ** 2

        prev = None
        done = 0
        for it in range(steps):
            for q in range(3):
                wv = ops[q](v[q])
                lam[q] = np.linalg.norm(wv)
                v[q] = wv / lam[q]
            done = it + 1
            if tol > 0 and done % POWER_CHECK == 0:
                cur = scal(*lam)
                if prev is not None and all(abs(c - p) <= tol * abs(c) for c, p in zip(cur, prev)):
                    break
                prev = cur
        alpha, beta, gamma = scal(*lam)
        self.set_scalings(alpha, beta, gamma)
        return alpha, beta, gamma, tuple(lam), done

    # ----- dense matrices ---------------------------------------------------
    def T(self):
        k = self.k
        return 1j * k * self.TA + self.TPhi / (1j * k)

    def Po(self):
        return self.P_LH / self.alpha + 1j * self.P_s / self.beta

    def Pm(self):
        return (self.ML_hat / self.alpha ** 2 + self.P_LH / self.gamma
                + self.MS_hat / self.beta ** 2)

    def system_direct(self):
        """A = P_o^H T^H P_m T P_o, formed as written in eq. NewFormulation."""
        Po, T, Pm = self.Po(), self.T(), self.Pm()
        return Po.conj().T @ T.conj().T @ Pm @ T @ Po

    def system_split(self):
        """Dense A from the cancellation-free application (column by column)."""
        N = self.top.N
        return self.apply(np.eye(N, dtype=np.complex128))

    # ----- cancellation-free application ------------------------------------
    def _left(self, wL, wS):
        """y = P_o^H T^H w for w = wL + wS, wL = P_mL(.) and wS = P_mS(.).

        T^H = -ik conj(T_A) + (i/k) conj(T_Phi).  Two products are identically
        zero and are dropped, so that no O(1/k) term meets an O(k) one:
        P_LH conj(T_Phi) (P_LH Sig = 0) and Sig^T P_mL (Sig^T Lam = 0 and
        Sig^T P_LH = 0).
        """
        k, al, be = self.k, self.alpha, self.beta
        Sig = self.top.Sigma
        zA = np.conj(self.TA) @ (wL + wS)
        vw = np.conj(self.V) @ (Sig.T @ wS)
        return (-(1j * k / al) * (self.P_LH @ zA)
                + self.P_s.T @ (-(k / be) * zA + (Sig @ vw) / (k * be)))

    def _middle(self, a, phi):
        """(wL, wS): P_mL a and P_mS (a + phi), phi in range(Sig).

        P_mL phi = 0 is dropped (Lam^T Sig = 0, P_LH Sig = 0).
        """
        al, be, ga = self.alpha, self.beta, self.gamma
        return (self.ML_hat @ a / al ** 2 + self.P_LH @ a / ga,
                self.MS_hat @ (a + phi) / be ** 2)

    def apply(self, x):
        """y = A x in cancellation-free order (x: [N] or [N, m])."""
        k, al, be = self.k, self.alpha, self.beta
        Sig = self.top.Sigma
        uS = self.P_s @ x
        uL = self.P_LH @ x
        # T P_o x = T_A((ik/alpha) u_L - (k/beta) u_S) + Sig V Sig^T u_S/(k beta);
        # T_Phi u_L = 0 is dropped.
        a = self.TA @ ((1j * k / al) * uL - (k / be) * uS)
        phi = Sig @ (self.V @ (Sig.T @ uS)) / (k * be)
        return self._left(*self._middle(a, phi))

    def rhs(self, e):
        """b = -P_o^H T^H P_m e (e: [N] or [N, m])."""
        al, be, ga = self.alpha, self.beta, self.gamma
        wL = self.ML_hat @ e / al ** 2 + self.P_LH @ e / ga
        wS = self.MS_hat @ e / be ** 2
        return -self._left(wL, wS)

    def recover(self, i):
        """j = P_o i (eq. NewFormulation)."""
        return self.P_LH @ i / self.alpha + 1j * (self.P_s @ i) / self.beta

    def rhs_split(self, s, e1):
        """b = -P_o^H T^H P_m e for e = Sigma s + e1 (rhs.planewave_split),
        without forming e: the static part Sigma s lies in the range of
        Sigma, where P_mL vanishes (Lam^T Sig = 0, P_LH Sig = 0) and
        P_mS Sigma s = Sig L^+ G_pp^-1 (s - mean s)/beta^2 (L^+ L = I - 1 1^T/C).
        So the O(1) static part never meets the O(k) loop part of e1."""
        al, be, ga = self.alpha, self.beta, self.gamma
        Sig = self.top.Sigma
        sm = np.asarray(s) - np.mean(s, axis=0)              # s [C] or [C, m]
        wL = self.ML_hat @ e1 / al ** 2 + self.P_LH @ e1 / ga
        wS = (self.MS_hat @ e1 + Sig @ (self.Lp @ (self.Gpp_inv @ sm))) / be ** 2
        return -self._left(wL, wS)

    def recover_split(self, i):
        """(j_loop, j_star) = (P_LH i/alpha, i P_s i/beta): the two parts of
        j = P_o i kept apart (at very low k the star part is O(k) relative to
        the loop part and would be lost in their sum)."""
        return self.P_LH @ i / self.alpha, 1j * (self.P_s @ i) / self.beta


POWER_CHECK = 5  # steps between convergence checks of the power iteration


def power_norm(op, start, steps):
    """2-norm of a Hermitian PSD operator: ``steps`` power iterations.

    v0 = start/|start|; each step w = op(v), lam = |w|, v = w/lam; returns the
    last lam.
    """
    v = start / np.linalg.norm(start)
    lam = 0.0
    for _ in range(steps):
        wv = op(v)
        lam = np.linalg.norm(wv)
        v = wv / lam
    return lam


def cg(apply, b, tol, maxit):
    """Complex CG for an HPD operator (Sec. 3.4), x0 = 0.

    Stops when the recursive residual satisfies |r|/|b| <= tol; then the true
    residual |b - A x|/|b| is evaluated and CG restarts on it until that meets
    tol too (or maxit total iterations).  Returns (x, iterations, true rel.
    residual).
    """
    b = np.asarray(b, dtype=np.complex128)
    bn = np.linalg.norm(b)
    x = np.zeros_like(b)
    total = 0
    while True:
        r = b - apply(x) if total else b.copy()
        rel = np.linalg.norm(r) / bn
        if rel <= tol or total >= maxit:
            return x, total, rel
        p = r.copy()
        rho = np.vdot(r, r).real
        while total < maxit:
            q = apply(p)
            a = rho / np.vdot(p, q).real
            x = x + a * p
            r = r - a * q
            total += 1
            rho_new = np.vdot(r, r).real
            if np.sqrt(rho_new) / bn <= tol:
                break
            p = r + (rho_new / rho) * p
            rho = rho_new


def iteration_bound(cond, eps):
    """CG iteration bound of eq. Niter: ceil(1/2 sqrt(cond) log(2/eps))."""
    return int(np.ceil(0.5 * np.sqrt(cond) * np.log(2.0 / eps)))


def efie_condition(top, TA, V, k):
    """Condition number of the unpreconditioned EFIE matrix (Sec. 2):
    T = i k T_A + Sigma V Sigma^T/(i k), which is complex symmetric but not
    Hermitian, so cond(T) is the ratio of its largest and smallest singular
    values.  The paper's introduction states that it grows as (k h)^-2."""
    Sig = top.Sigma
    T = 1j * k * TA + (Sig @ V @ Sig.T) / (1j * k)
    sv = np.linalg.svd(T, compute_uv=False)
    return float(sv[0] / sv[-1])
