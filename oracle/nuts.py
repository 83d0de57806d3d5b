"""No-U-turn sampler and its warm-up adaptation (oracle, FP64).

Test infrastructure only (see oracle/__init__.py).

Section 2.2: the posterior is sampled with NUTS, a Hamiltonian Monte Carlo
method that grows each trajectory until it starts to turn back, with the step
size and a diagonal mass matrix adapted during warm-up.  The paper relies on an
existing implementation and prints no algorithm; this module follows the
published method:
  * trajectory doubling in a random direction, one leapfrog step per leaf
    (Hoffman & Gelman 2014, "The No-U-Turn Sampler", Sec. 3);
  * multinomial selection of the new state with weights exp(-H): uniform
    progressive sampling inside a new subtree, and a move to the subtree's
    candidate with probability min(1, W_subtree / W_tree) when the subtree is
    joined to the tree (Betancourt 2017, "A Conceptual Introduction to
    Hamiltonian Monte Carlo", Appendix A.3);
  * the generalised no-U-turn criterion: a (sub)tree with end momenta p-, p+
    and momentum sum rho (over all its leaves) is turning when
    (M^-1 p-) . rho <= 0 or (M^-1 p+) . rho <= 0 (Betancourt 2017, A.4.2),
    checked for the whole tree after every doubling and for every aligned
    power-of-two block of leaves inside a new subtree;
  * a subtree that turns or diverges (H - H0 > 1000) is discarded and the
    trajectory ends;
  * step-size adaptation by dual averaging (Hoffman & Gelman 2014, Sec. 3.2)
    towards a mean acceptance statistic of 0.8;
  * diagonal mass matrix from Welford variances over expanding windows.

Random numbers are inputs: z (standard normal, one per coordinate) gives the
momentum p = M^(1/2) z, and `uniforms` holds, per transition, max_depth
direction draws, then max_depth join draws, then one draw per leaf in the order
the leaves are made (2^max_depth - 1 of them).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .hmc import SCHEMES

DELTA_MAX = 1000.0


def n_uniforms(max_depth: int) -> int:
    """Uniform draws one transition consumes (direction, join, leaves)."""
    return 2 * max_depth + (1 << max_depth) - 1


def _logaddexp(a: float, b: float) -> float:
    if a == -math.inf:
        return b
    if b == -math.inf:
        return a
    m = max(a, b)
    return m + math.log(math.exp(a - m) + math.exp(b - m))


def _turning(minv, p_minus, p_plus, rho, margins=None) -> bool:
    a = float(np.dot(minv * p_minus, rho))
    b = float(np.dot(minv * p_plus, rho))
    if margins is not None:
        nr = np.linalg.norm(rho)
        margins.append(min(abs(a) / (np.linalg.norm(minv * p_minus) * nr + 1e-300),
                           abs(b) / (np.linalg.norm(minv * p_plus) * nr + 1e-300)))
    return a <= 0.0 or b <= 0.0


@dataclass
class Transition:
    q: np.ndarray          # new state
    grad: np.ndarray       # dU/dq at the new state
    potential: float       # U at the new state
    accept_stat: float     # mean of min(1, exp(H0 - H)) over every leaf made
    depth: int             # doublings joined to the tree
    n_leapfrog: int        # leaves made (leapfrog steps taken)
    diverging: bool
    h0: float
    # smallest distance of any random or sign decision from its threshold:
    # |uniform - probability| for candidate choices and joins, and
    # |(M^-1 p) . rho| / (|M^-1 p| |rho|) for U-turn checks (how far a result
    # computed with a different rounding can move before a decision flips)
    margin_choice: float = math.inf
    margin_turn: float = math.inf


def transition(pot_grad, q0, z, minv, eps, uniforms, max_depth, start=None, scheme="leapfrog"):
    """One NUTS transition from q0.  `pot_grad(q) -> (U, dU/dq)` on flat float64
    vectors; minv is the diagonal inverse mass matrix; `start` optionally holds
    (U, dU/dq) at q0.  Each leaf is one step of a splitting scheme of
    oracle.hmc.SCHEMES (a symmetric, volume-preserving step, so the tree
    stays a valid NUTS trajectory)."""
    kicks, drifts = SCHEMES[scheme]
    q0 = np.asarray(q0, dtype=np.float64)
    minv = np.broadcast_to(np.asarray(minv, dtype=np.float64), q0.shape)
    u0, g0 = start if start is not None else pot_grad(q0)
    p0 = np.asarray(z, dtype=np.float64) / np.sqrt(minv)
    h0 = u0 + 0.5 * float(np.sum(minv * p0 * p0))
    ends = {-1: (q0, p0, g0), +1: (q0, p0, g0)}
    cand = (q0, g0, u0)
    log_w = 0.0                      # log of the tree's weight, relative to exp(-H0)
    rho = p0.copy()
    acc_sum, n_leaf, depth, diverging = 0.0, 0, 0, False
    m_choice, m_turn = [math.inf], [math.inf]
    for j in range(max_depth):
        v = 1 if uniforms[j] >= 0.5 else -1
        q, p, g = ends[v]
        leaves_p, log_ws = [], -math.inf
        cand_s = None
        stop = False
        for k in range(1 << j):
            for a_i, b_i in zip(kicks, drifts):
                p = p - a_i * v * eps * g
                q = q + b_i * v * eps * minv * p
                u_pot, g = pot_grad(q)
            p = p - kicks[-1] * v * eps * g
            h = u_pot + 0.5 * float(np.sum(minv * p * p))
            n_leaf += 1
            acc_sum += min(1.0, math.exp(min(0.0, h0 - h)))
            if not (h - h0 <= DELTA_MAX):      # also catches NaN energies
                diverging = stop = True
                break
            log_ws = _logaddexp(log_ws, h0 - h)
            r, prob = uniforms[2 * max_depth + (1 << j) - 1 + k], math.exp((h0 - h) - log_ws)
            if k > 0:
                m_choice.append(abs(r - prob))
            if r < prob:
                cand_s = (q, g, u_pot)
            leaves_p.append(p)
            # every aligned block of 2, 4, ... leaves that ends here
            size = 2
            while (k + 1) % size == 0:
                blk = leaves_p[k + 1 - size:k + 1]
                if _turning(minv, blk[0], blk[-1], np.sum(blk, axis=0), m_turn):
                    stop = True
                    break
                size *= 2
            if stop:
                break
        if stop:
            break
        r, prob = uniforms[max_depth + j], math.exp(min(0.0, log_ws - log_w))
        if prob < 1.0:
            m_choice.append(abs(r - prob))
        if r < prob:
            cand = cand_s
        log_w = _logaddexp(log_w, log_ws)
        ends[v] = (q, p, g)
        rho = rho + np.sum(leaves_p, axis=0)
        depth = j + 1
        if _turning(minv, ends[-1][1], ends[+1][1], rho, m_turn):
            break
    return Transition(cand[0], cand[1], cand[2], acc_sum / max(n_leaf, 1), depth, n_leaf, diverging, h0,
                      min(m_choice), min(m_turn))


class DualAveraging:
    """Step-size adaptation of Hoffman & Gelman 2014, Sec. 3.2 (after Nesterov
    2009): log eps_t = mu - sqrt(t)/gamma * Hbar_t with
    Hbar_t = (1 - 1/(t+t0)) Hbar_{t-1} + (delta - a_t)/(t+t0), and the averaged
    log eps_bar_t = t^-kappa log eps_t + (1 - t^-kappa) log eps_bar_{t-1};
    mu = log(10 eps_0)."""

    def __init__(self, eps0, target=0.8, gamma=0.05, t0=10.0, kappa=0.75):
        self.mu = math.log(10.0 * eps0)
        self.target, self.gamma, self.t0, self.kappa = target, gamma, t0, kappa
        self.t = 0
        self.h_bar = 0.0
        self.log_eps_bar = 0.0

    def update(self, accept_stat) -> float:
        self.t += 1
        t = self.t
        w = 1.0 / (t + self.t0)
        self.h_bar = (1.0 - w) * self.h_bar + w * (self.target - accept_stat)
        log_eps = self.mu - math.sqrt(t) / self.gamma * self.h_bar
        eta = t ** (-self.kappa)
        self.log_eps_bar = eta * log_eps + (1.0 - eta) * self.log_eps_bar
        return math.exp(log_eps)

    def final(self) -> float:
        return math.exp(self.log_eps_bar)


class Welford:
    """Running mean and sum of squared deviations (Welford 1962)."""

    def __init__(self, dim):
        self.n = 0
        self.mean = np.zeros(dim)
        self.m2 = np.zeros(dim)

    def add(self, x):
        self.n += 1
        d = x - self.mean
        self.mean = self.mean + d / self.n
        self.m2 = self.m2 + d * (x - self.mean)

    def variance(self):
        return self.m2 / (self.n - 1)


def regularized_inverse_mass(var, n):
    """Diagonal M^-1 from a window's sample variance, shrunk towards 1e-3 with
    weight 5/(n+5) (the shrinkage used by Stan's windowed adaptation)."""
    return (n / (n + 5.0)) * var + 1e-3 * (5.0 / (n + 5.0))


def window_ends(n_warmup, init_buffer=75, term_buffer=50, base_window=25):
    """Iterations (1-based counts) after which a mass-matrix window closes:
    windows of base_window, 2 base_window, ... between an initial and a
    terminal buffer, the last window stretched to the terminal buffer."""
    ends = []
    if n_warmup < init_buffer + term_buffer + base_window:
        return ends
    start, size = init_buffer, base_window
    last = n_warmup - term_buffer
    while start + size <= last:
        nxt = start + size
        if nxt + 2 * size > last:
            nxt = last
        ends.append(nxt)
        start, size = nxt, 2 * size
    return ends
