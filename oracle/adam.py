"""Adam optimiser (test infrastructure; see oracle/__init__).

Sec. 3.4 ("Training") trains with Adam at learning rate 1e-3.  The update is
Kingma & Ba 2014, Algorithm 1, with the remaining constants at their usual
defaults (beta1 0.9, beta2 0.999, epsilon 1e-8, no weight decay):
    m <- b1 m + (1 - b1) g
    v <- b2 v + (1 - b2) g^2
    theta <- theta - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
with t the 1-based step count.  float64 state.
"""

from __future__ import annotations

import numpy as np


class Adam:
    def __init__(self, n: int, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999,
                 eps: float = 1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, theta, g) -> np.ndarray:
        g = np.asarray(g, dtype=np.float64)
        self.t += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * g
        self.v = self.b2 * self.v + (1.0 - self.b2) * g * g
        mhat = self.m / (1.0 - self.b1 ** self.t)
        vhat = self.v / (1.0 - self.b2 ** self.t)
        return np.asarray(theta, dtype=np.float64) - self.lr * mhat / (np.sqrt(vhat) + self.eps)
