"""Anderson mixing (Appendix D).

With f_k = vhat_k - v_k, S_k = [v_i - v_{i-1}] and Y_k = [f_i - f_{i-1}] over
the last m steps and C_{k-1} = -zeta I:
  v_{k+1} = v_k + zeta f_k - (S_k + zeta Y_k) (Y_k^T Y_k)^{-1} Y_k^T f_k.
gamma = (Y^T Y)^{-1} Y^T f is the least-squares solution of Y gamma ~ f and is
computed here by QR.  With no history (k = 0) the step is v + zeta f.
Ill-conditioned history: the oldest columns are dropped until the condition
number of Y^T Y is below 1e12.
"""
import numpy as np


class Anderson:
    def __init__(self, m: int, zeta: float, cond_max: float = 1e12):
        self.m, self.zeta, self.cond_max = m, zeta, cond_max
        self.S, self.Y = [], []
        self.v_prev = self.f_prev = None

    def step(self, v: np.ndarray, f: np.ndarray) -> np.ndarray:
        v = v.ravel().astype(np.float64)
        f = f.ravel().astype(np.float64)
        if self.v_prev is not None and self.m > 0:
            self.S.append(v - self.v_prev)
            self.Y.append(f - self.f_prev)
            del self.S[:-self.m]
            del self.Y[:-self.m]
        self.v_prev, self.f_prev = v.copy(), f.copy()
        out = v + self.zeta * f
        while self.Y:
            Y = np.stack(self.Y, 1)
            ev = np.linalg.eigvalsh(Y.T @ Y)
            if ev[0] > 0 and ev[-1] / ev[0] < self.cond_max:
                break
            self.S.pop(0)
            self.Y.pop(0)
        if self.Y:
            Y = np.stack(self.Y, 1)
            S = np.stack(self.S, 1)
            q, r = np.linalg.qr(Y)
            gamma = np.linalg.solve(r, q.T @ f)
            out = out - (S + self.zeta * Y) @ gamma
        return out
