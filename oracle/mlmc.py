"""Multilevel Monte Carlo estimator (oracle side), Sec. 2.2-2.3.

  Y_0 = Q_0,  Y_l = Q_l - Q_{l-1}, the two meshes of a level-l sample sharing
  one draw xi(l, i) (eq. mlmc_average and the sentence after it)
  Qtilde_L = sum_l mean(Y_l)                                 (eq. mlmc_average)
  V(Y_l)  = (1/N_l) sum_i (Y_l^i - mean(Y_l))^2  -- note 1/N (eq. sample_variance)
  V(Qtilde_L) = sum_l V(Y_l) / N_l                           (Sec. 2.2)
  N_l = ceil(2 eps^-2 sqrt(V_l / C_l) sum_i sqrt(V_i C_i))   (eq. mlmc_num_samples)
  L   = ceil(log_s(sqrt(2) c / eps) / alpha)                 (eq. mlmc_num_levels)
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import numpy as np

from . import fe, field, pcg, rng


def solve_qoi(n: int, kap: np.ndarray, qoi: int, rtol: float, max_iter: int, b=None):
    """Q(u_h) for one sample: Jacobi-PCG on the assembled operator; f = 1 unless b is given."""
    A = fe.assemble(n, kap)
    if b is None:
        b = fe.load_constant(n)
    u, it, rel = pcg.jacobi_pcg(A, b, rtol, max_iter)
    return float(fe.qoi_weights(n, qoi) @ u), it, rel, u


def sample_level(wl, level: int, first: int, count: int, rtol=None, max_iter=None,
                 common_random_numbers: bool = False):
    """Per-sample (Y, Q_fine, Q_coarse, iterations_fine) for one level.

    common_random_numbers: draw xi with level 0 in the counter for every level
    (test-only mode used by the telescoping identity).
    """
    rtol = wl.rtol if rtol is None else rtol
    max_iter = wl.max_iter if max_iter is None else max_iter
    lv = 0 if common_random_numbers else level
    xi = rng.draw_xi(wl.seed, lv, first, count, wl.n_modes)
    nf = wl.n(level)
    kf = field.kappa(nf, wl.corr_len, wl.sigma2, wl.n_modes, xi)
    kc = field.kappa(nf // 2, wl.corr_len, wl.sigma2, wl.n_modes, xi) if level > 0 else None
    forced = getattr(wl, "forcing", 0) == 1
    if forced:   # f = exp(g_f): the KLE of the log-field with its own coefficients (stream 2)
        xif = rng.draw_xi(wl.seed, lv, first, count, wl.n_modes, stream=2)
        ff = field.kappa(nf, wl.corr_len, wl.sigma2, wl.n_modes, xif)
        fc = field.kappa(nf // 2, wl.corr_len, wl.sigma2, wl.n_modes, xif) if level > 0 else None
    Y = np.empty(count); Qf = np.empty(count); Qc = np.zeros(count); its = np.empty(count, dtype=np.int64)
    for s in range(count):
        bf = fe.load_elements(nf, ff[s]) if forced else None
        Qf[s], its[s], _, _ = solve_qoi(nf, kf[s], wl.qoi, rtol, max_iter, bf)
        if level > 0:
            bc = fe.load_elements(nf // 2, fc[s]) if forced else None
            Qc[s], _, _, _ = solve_qoi(nf // 2, kc[s], wl.qoi, rtol, max_iter, bc)
        Y[s] = Qf[s] - Qc[s]
    return Y, Qf, Qc, its


@dataclasses.dataclass
class RunningStats:
    """Count, mean and sum of squared deviations (Welford, in sample order)."""
    n: int = 0
    mean: float = 0.0
    m2: float = 0.0

    def push(self, y: float):
        self.n += 1
        d = y - self.mean
        self.mean += d / self.n
        self.m2 += d * (y - self.mean)

    def merge(self, other: "RunningStats") -> "RunningStats":
        """Chan, Golub and LeVeque pairwise combination."""
        n = self.n + other.n
        if n == 0:
            return RunningStats()
        d = other.mean - self.mean
        mean = self.mean + d * other.n / n
        m2 = self.m2 + other.m2 + d * d * self.n * other.n / n
        return RunningStats(n, mean, m2)

    @property
    def var(self) -> float:
        """eq. sample_variance: 1/N normalisation."""
        return self.m2 / self.n if self.n else 0.0


def estimator(stats: Sequence[RunningStats]):
    """(Qtilde, per-level V(Y_l), V(Qtilde) = sum V_l / N_l)."""
    qt = sum(s.mean for s in stats)
    v = [s.var for s in stats]
    vq = sum(s.var / s.n for s in stats if s.n)
    return qt, v, vq


def optimal_samples(var: Sequence[float], cost: Sequence[float], eps: float,
                    extra_fraction: float = 0.0) -> List[int]:
    """eq. mlmc_num_samples, each N_l scaled by (1 + extra_fraction) before the
    ceiling (Sec. 2.3 draws a fraction more than the formula asks for)."""
    tot = sum(math.sqrt(v * c) for v, c in zip(var, cost))
    return [int(math.ceil(2.0 / (eps * eps) * math.sqrt(v / c) * tot * (1.0 + extra_fraction)))
            for v, c in zip(var, cost)]


def num_levels(c: float, alpha: float, eps: float, s: float = 2.0) -> int:
    """eq. mlmc_num_levels."""
    return int(math.ceil(math.log(math.sqrt(2.0) * c / eps, s) / alpha))


def level_cost(wl, level: int) -> float:
    """Deterministic cost model: interior unknowns solved for one Y_l sample."""
    n = wl.n(level)
    return float((n - 1) ** 3 + ((n // 2 - 1) ** 3 if level > 0 else 0))


def run_mlmc(wl, n_per_level: Sequence[int]):
    """Plain MLMC with fixed N_l; returns (Qtilde, V_l list, V(Qtilde), stats, Ys)."""
    stats, ys = [], []
    for lvl, N in enumerate(n_per_level):
        Y, _, _, _ = sample_level(wl, lvl, 0, N)
        st = RunningStats()
        for y in Y:
            st.push(float(y))
        stats.append(st)
        ys.append(Y)
    qt, v, vq = estimator(stats)
    return qt, v, vq, stats, ys


def estimate(wl, eps: float, n_pilot: int, max_rounds: int = 3, extra_fraction: float = 0.0, sampler=None,
             cost=None, n_fixed: Sequence[int] = None):
    """Pilot, optimal allocation (eq. mlmc_num_samples) and top-up on the fixed
    level set.  Round 0 draws n_pilot samples per level; each later round
    tops every level up to max(N_l, n_pilot), N_l from the current 1/N
    variances (eq. sample_variance) and the costs C_l, until no level grows or
    max_rounds allocations were made.  A level's samples continue its index
    range (sample i of level l is always the same draw).
    `sampler(level, first, count)` returns the Y values (default: the FE path
    of sample_level); `cost(level)` the cost of one Y_l (default: the
    deterministic DOF model).  n_fixed: plain MLMC with caller-given N_l
    (Sec. 2.2): every level is sampled to n_fixed[l], no pilot or allocation.
    Returns (N_l list, Qtilde, V(Qtilde), stats)."""
    if sampler is None:
        sampler = lambda l, first, count: sample_level(wl, l, first, count)[0]
    if cost is None:
        cost = lambda l: level_cost(wl, l)
    L = wl.levels
    stats = [RunningStats() for _ in range(L)]

    def top_up(target):
        more = False
        for l in range(L):
            have = stats[l].n
            if target[l] > have:
                more = True
                for y in sampler(l, have, target[l] - have):
                    stats[l].push(float(y))
        return more

    if n_fixed is not None:
        top_up(list(n_fixed))
    else:
        target = [n_pilot] * L
        for rnd in range(max_rounds + 1):
            more = top_up(target)
            if (not more and rnd > 0) or rnd == max_rounds:
                break
            want = optimal_samples([s.var for s in stats], [cost(l) for l in range(L)], eps, extra_fraction)
            grow = False
            for l in range(L):
                if max(want[l], n_pilot) > target[l]:
                    target[l] = max(want[l], n_pilot)
                    grow = True
            if not grow:
                break
    qt, v, vq = estimator(stats)
    return [s.n for s in stats], qt, vq, stats


def fit_decay(values: Sequence[float], levels: Sequence[int], s: float = 2.0):
    """Least-squares fit of values_l ~ c s^(-r l): the slope of log_s(values)
    against l (Sec. 2.3: c and alpha of eq. mlmc_num_levels are estimated from
    the level means, the decay of the level variances likewise).  Returns
    (c, r)."""
    x = [float(l) for l in levels]
    y = [math.log(v) / math.log(s) for v in values]
    xm = sum(x) / len(x)
    ym = sum(y) / len(y)
    sxx = sum((a - xm) * (a - xm) for a in x)
    sxy = sum((a - xm) * (b - ym) for a, b in zip(x, y))
    r = -sxy / sxx
    c = s ** (ym + r * xm)
    return c, r


def _rate(values: Sequence[float], l_max: int, default: float, lo: float, hi: float, s: float):
    """(c, r) of values_l ~ c s^(-r l) over l = 1..l_max: fitted when there are
    two or more levels (r clamped to [lo, hi], c refitted for the clamped r),
    else r = default through the single point."""
    lv = list(range(1, l_max + 1))
    vals = [max(abs(values[l]), 1e-300) for l in lv]
    if len(lv) >= 2:
        c, r = fit_decay(vals, lv, s)
        if lo <= r <= hi:
            return c, r
        r = min(max(r, lo), hi)
    else:
        r = default
    logc = sum(math.log(v) / math.log(s) + r * l for v, l in zip(vals, lv)) / len(lv)
    return s ** logc, r


def estimate_adaptive(wl, eps: float, l0: int, n_pilot: int, max_rounds: int = 10, alpha0: float = 2.0,
                      beta0: float = 4.0, extra_fraction: float = 0.0, sampler=None, cost=None, s: float = 2.0):
    """Adaptive MLMC (Sec. 2.3 and the adaptive loop of Alg. dyn_par_sched),
    read as a do-while loop: sample every level up to its target, estimate the
    error e^2 = bias^2 + V(Qtilde) (eq. mlmc_error), stop when e <= eps; else
    update L by eq. mlmc_num_levels and the targets by eq. mlmc_num_samples,
    and repeat.

    Readings (the paper leaves them open): the level means fit
    |mean(Y_l)| ~ c s^(-alpha l) over l = 1..L (alpha = alpha0 with one level,
    else least squares clamped to [0.5, 4]); the bias of Qtilde_L is the
    geometric tail sum_{k>L} c s^(-alpha k) = c s^(-alpha L) / (s^alpha - 1),
    so eq. mlmc_num_levels takes c / (s^alpha - 1); L only grows and stays
    below the number of configured meshes; the variances of levels not yet
    sampled follow V_l ~ cV s^(-beta l) fitted like alpha (beta0 with one
    level, clamp [0.5, 8]); new levels get at least n_pilot samples; targets
    never decrease.  `sampler(level, first, count)` returns Y values (default:
    the FE path of sample_level); `cost(level)` the cost of one Y_l (default:
    the deterministic DOF model).
    Returns a dict with L, n_per_level, qtilde, var_qtilde, bias, err, alpha,
    beta, rounds, stats."""
    if sampler is None:
        sampler = lambda l, first, count: sample_level(wl, l, first, count)[0]
    if cost is None:
        cost = lambda l: level_cost(wl, l)
    M = wl.levels
    if not 1 <= l0 < M:
        raise ValueError("need 1 <= l0 < number of levels")
    L = l0
    stats = [RunningStats() for _ in range(M)]
    target = [n_pilot] * (L + 1) + [0] * (M - L - 1)
    alpha = beta = bias = err = float("nan")
    rounds = 0
    for rnd in range(max_rounds + 1):
        rounds = rnd + 1
        for l in range(L + 1):
            have = stats[l].n
            if target[l] > have:
                for y in sampler(l, have, target[l] - have):
                    stats[l].push(float(y))
        means = [st.mean for st in stats]
        var = [st.var for st in stats]
        cY, alpha = _rate(means, L, alpha0, 0.5, 4.0, s)
        cV, beta = _rate(var, L, beta0, 0.5, 8.0, s)
        tail = s ** alpha - 1.0
        bias = cY * s ** (-alpha * L) / tail
        vq = sum(var[l] / stats[l].n for l in range(L + 1))
        err = math.sqrt(bias * bias + vq)
        if err <= eps or rnd == max_rounds:
            break
        L_new = min(M - 1, max(L, num_levels(cY / tail, alpha, eps, s)))
        V = [var[l] if l <= L else cV * s ** (-beta * l) for l in range(L_new + 1)]
        C = [cost(l) for l in range(L_new + 1)]
        tot = sum(math.sqrt(v * c) for v, c in zip(V, C))
        grow = L_new > L
        for l in range(L_new + 1):
            want = int(math.ceil(2.0 / (eps * eps) * math.sqrt(V[l] / C[l]) * tot * (1.0 + extra_fraction)))
            want = max(want, n_pilot)
            if want > target[l]:
                target[l] = want
                grow = True
        L = L_new
        if not grow:
            break
    qt = sum(stats[l].mean for l in range(L + 1))
    vq = sum(stats[l].var / stats[l].n for l in range(L + 1))
    return dict(L=L, n_per_level=[stats[l].n for l in range(L + 1)], qtilde=qt, var_qtilde=vq, bias=bias, err=err,
                alpha=alpha, beta=beta, rounds=rounds, stats=stats[:L + 1])
