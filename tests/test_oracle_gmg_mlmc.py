"""Pins for the multigrid pieces and the MLMC statistics of the oracle."""
import math

import numpy as np
import pytest

from oracle import fe, gmg, mlmc, rng
from workloads import C1, Workload, element_field, grid_vector


def test_coarsen_kappa_mean():
    n = 8
    kap = element_field(n, 2, seed=1)
    kc = gmg.coarsen_kappa(n, kap)
    # element (1, 2, 3) of the n/2 grid has children (2..3, 4..5, 6..7)
    want = np.mean([kap[1, x + n * (y + n * z)] for x in (2, 3) for y in (4, 5) for z in (6, 7)])
    assert kc[1, 1 + 4 * (2 + 4 * 3)] == pytest.approx(want, rel=1e-15)
    assert np.all(gmg.coarsen_kappa(n, np.full(n ** 3, 2.5)) == 2.5)


@pytest.mark.parametrize("n", [4, 8, 16])
def test_galerkin_identity_constant_kappa(n):
    # nested conforming spaces: P^T A_h P = A_2h exactly for constant kappa
    c = 1.7
    Af = fe.assemble(n, np.full(n ** 3, c))
    Ac = fe.assemble(n // 2, np.full((n // 2) ** 3, c))
    P = gmg.prolongation(n)
    G = (P.T @ Af @ P).toarray()
    assert np.abs(G - Ac.toarray()).max() <= 1e-14 * np.abs(Ac.toarray()).max()


def test_prolongation_reproduces_coarse_trilinear():
    # a function trilinear on each coarse cell and zero on the boundary
    n = 8
    nc = n // 2
    cg = fe.interior_ijk(nc)
    uc = grid_vector(nc, 1, seed=2)[0]
    uf = gmg.prolongation(n) @ uc
    full = np.zeros((nc + 1,) * 3)
    full[cg[:, 2], cg[:, 1], cg[:, 0]] = uc
    for i, j, k in fe.interior_ijk(n)[::7]:
        X = np.array([i, j, k]) / 2.0
        lo = np.floor(X).astype(int)
        t = X - lo
        val = 0.0
        for a in range(8):
            o = np.array([a & 1, (a >> 1) & 1, (a >> 2) & 1])
            p = np.minimum(lo + o, nc)
            w = np.prod(np.where(o == 1, t, 1 - t))
            val += w * full[p[2], p[1], p[0]]
        assert uf[fe.interior_index(n, i, j, k)] == pytest.approx(val, abs=1e-15)


def test_chebyshev_matches_polynomial():
    n = 4
    kap = element_field(n, 1, seed=4)[0]
    A = fe.assemble(n, kap)
    dinv = 1.0 / A.diagonal()
    xstar = grid_vector(n, 1, seed=5)[0]
    b = A @ xstar
    x0 = grid_vector(n, 1, seed=6)[0]
    lo, hi = 0.5, 2.0
    # symmetric form S = D^-1/2 A D^-1/2; e_s = D^-1/2 p(S) D^1/2 e_0
    d = np.sqrt(A.diagonal())
    S = A.toarray() / d[:, None] / d[None, :]
    lam, V = np.linalg.eigh(S)
    for deg in (1, 2, 3, 4):
        xs = gmg.chebyshev(A, dinv, b, x0, deg, lo, hi)
        p = gmg.chebyshev_polynomial(lam, deg, lo, hi)
        e = (V @ (p * (V.T @ (d * (xstar - x0))))) / d
        assert np.abs((xstar - xs) - e).max() < 1e-12 * np.abs(xstar - x0).max()


def test_vcycle_symmetric_positive_contracting():
    n = 8
    kap = element_field(n, 1, seed=7, spread=1.5)[0]
    H = gmg.Hierarchy(n, kap)
    r1, r2 = grid_vector(n, 2, seed=8)
    v1 = H.vcycle(r1, 2, 4.0, 2.0)
    v2 = H.vcycle(r2, 2, 4.0, 2.0)
    assert abs(v1 @ r2 - v2 @ r1) <= 1e-12 * abs(v1 @ r2)
    assert v1 @ r1 > 0
    # two-grid-like contraction of I - B A on a random error
    A = H.As[0]
    e = r1.copy()
    for _ in range(3):
        e = e - H.vcycle(A @ e, 2, 4.0, 2.0)
    assert np.linalg.norm(e) < 0.05 * np.linalg.norm(r1)


def test_welford_and_chan_against_two_pass():
    y = np.random.default_rng(9).standard_normal(1001) * 3 + 0.7
    s = mlmc.RunningStats()
    for v in y:
        s.push(v)
    assert s.mean == pytest.approx(y.mean(), rel=1e-14)
    assert s.var == pytest.approx(np.mean((y - y.mean()) ** 2), rel=1e-13)   # 1/N
    a, b = mlmc.RunningStats(), mlmc.RunningStats()
    for v in y[:400]:
        a.push(v)
    for v in y[400:]:
        b.push(v)
    m = a.merge(b)
    assert m.n == 1001 and m.mean == pytest.approx(s.mean, rel=1e-14)
    assert m.m2 == pytest.approx(s.m2, rel=1e-13)


def test_optimal_allocation_is_the_lagrange_optimum():
    V = [4e-4, 3e-5, 2e-6, 1.5e-7]
    C = [1.0, 8.0, 64.0, 512.0]
    eps = 1e-3
    N = mlmc.optimal_samples(V, C, eps)
    # continuous optimum: N_l = 2 eps^-2 sqrt(V_l/C_l) sum sqrt(V C); it meets
    # sum V_l / N_l = eps^2 / 2 exactly before the ceiling
    cont = [2 / eps ** 2 * math.sqrt(v / c) * sum(math.sqrt(a * b) for a, b in zip(V, C)) for v, c in zip(V, C)]
    assert N == [math.ceil(x) for x in cont]
    assert sum(v / x for v, x in zip(V, cont)) == pytest.approx(eps ** 2 / 2, rel=1e-12)
    assert sum(v / x for v, x in zip(V, N)) <= eps ** 2 / 2
    # any feasible perturbation costs more
    base = sum(c * x for c, x in zip(C, cont))
    for l in range(4):
        pert = list(cont)
        pert[l] *= 1.1
        other = (l + 1) % 4
        # keep the variance constraint by adjusting another level
        rest = eps ** 2 / 2 - sum(V[i] / pert[i] for i in range(4) if i != other)
        pert[other] = V[other] / rest
        assert sum(c * x for c, x in zip(C, pert)) > base


def test_num_levels_formula():
    # with alpha = 2, s = 2: L = ceil(log2(sqrt 2 c / eps) / 2)
    assert mlmc.num_levels(1.0, 2.0, 1e-3) == math.ceil(math.log2(math.sqrt(2) * 1e3) / 2)


def test_sample_scaling_law_table():
    # Sec. 5: N_l proportional to exp(Gamma log(s) (L - l)), Gamma = 4, s = 2,
    # L = 2; the paper's Table (sample sizes by level) lists 1024, 64, 4.
    table = [int(x) for x in open(__file__.replace("test_oracle_gmg_mlmc.py", "golden/sample_sizes_by_level.txt"))
             .read().split("#")[0].split()]
    law = [math.exp(4 * math.log(2.0) * (2 - l)) for l in range(3)]
    assert [round(4 * x) for x in law] == table


def test_telescoping_identity_common_random_numbers():
    # with common random numbers and equal N_l, sum_l mean(Y_l) = mean(Q_L)
    wl = Workload("tele", n0=2, levels=3, sigma2=1.0, corr_len=0.5, n_modes=8, rtol=1e-12, solver=1)
    N = 6
    ys, qL = [], None
    for lvl in range(3):
        Y, Qf, Qc, _ = mlmc.sample_level(wl, lvl, 0, N, common_random_numbers=True)
        ys.append(Y)
        if lvl == 2:
            qL = Qf
    tel = sum(y.mean() for y in ys)
    assert tel == pytest.approx(qL.mean(), rel=1e-14)


def test_c1_variance_decays_with_level():
    qt, v, vq, stats, ys = mlmc.run_mlmc(C1, (40, 20, 8))
    assert v[1] < v[0] / 4 and v[2] < v[1] / 4
    assert 0.0 < qt < 0.05
    assert vq == pytest.approx(sum(s.var / s.n for s in stats))


# ---------------------------------------------------------------- adaptive MLMC
# The adaptive loop (Sec. 2.3, adaptive loop of Alg. dyn_par_sched) pinned on a
# synthetic level model whose means and variances decay at known rates, so the
# level eq. mlmc_num_levels must choose and the allocation of
# eq. mlmc_num_samples are fixed by the model rather than by the FE path.

class _LevelSet:
    def __init__(self, levels):
        self.levels = levels


def _model(c=0.1, alpha=2.0, v=1e-4, beta=4.0, s=2.0, q0=0.5):
    def mean(l):
        return q0 if l == 0 else c * s ** (-alpha * l)

    def sd(l):
        return math.sqrt(v * s ** (-beta * l))

    def sampler(l, first, count):
        return np.array([mean(l) + sd(l) * np.random.default_rng([l, first + i]).standard_normal()
                         for i in range(count)])
    return sampler


def test_fit_decay_recovers_geometric_rates():
    for c, r in ((3.0, 2.0), (0.02, 1.3), (5e-5, 4.5)):
        lv = [1, 2, 3, 4]
        cc, rr = mlmc.fit_decay([c * 2.0 ** (-r * l) for l in lv], lv)
        assert rr == pytest.approx(r, rel=1e-12) and cc == pytest.approx(c, rel=1e-12)


def test_rate_clamped_and_single_level():
    # a flat sequence clamps to the lower bound; c then fits the points for it
    c, r = mlmc._rate([0.0, 1.0, 1.0, 1.0], 3, 2.0, 0.5, 4.0, 2.0)
    assert r == 0.5 and c == pytest.approx(2.0 ** (0.5 * 2), rel=1e-12)
    # one difference level: the default rate through that point
    c, r = mlmc._rate([0.0, 0.3], 1, 2.0, 0.5, 4.0, 2.0)
    assert r == 2.0 and c == pytest.approx(0.3 * 4.0, rel=1e-12)


def test_adaptive_loop_finds_the_level_of_a_known_model():
    c, alpha, eps = 0.1, 2.0, 1e-3
    cost = lambda l: 8.0 ** l
    r = mlmc.estimate_adaptive(_LevelSet(7), eps, 1, 16, max_rounds=10, sampler=_model(c, alpha), cost=cost)
    # the first level whose tail bias c s^-aL / (s^a - 1) is within eps / sqrt(2)
    lstar = min(L for L in range(1, 7) if c * 2.0 ** (-alpha * L) / (2.0 ** alpha - 1) <= eps / math.sqrt(2))
    assert lstar == 3
    assert r["L"] == lstar and r["err"] <= eps
    assert r["alpha"] == pytest.approx(alpha, abs=0.1) and r["beta"] == pytest.approx(4.0, abs=0.5)
    assert r["bias"] == pytest.approx(c * 2.0 ** (-alpha * lstar) / 3.0, rel=0.1)
    # the statistical half meets eps^2 / 2 (eq. mlmc_num_samples) up to the estimation noise
    assert r["var_qtilde"] <= 1.2 * eps ** 2 / 2
    # the telescoping sum estimates E(Q_L) of the model
    want = 0.5 + sum(c * 2.0 ** (-alpha * l) for l in range(1, lstar + 1))
    assert abs(r["qtilde"] - want) <= 4 * math.sqrt(r["var_qtilde"])
    # N_l is eq. mlmc_num_samples on the final variances (targets only grow)
    V = [s.var for s in r["stats"]]
    C = [cost(l) for l in range(lstar + 1)]
    tot = sum(math.sqrt(v * cc) for v, cc in zip(V, C))
    for l in range(lstar + 1):
        n_eq = 2.0 / eps ** 2 * math.sqrt(V[l] / C[l]) * tot
        assert r["n_per_level"][l] >= min(n_eq, 16) * 0.8


def test_adaptive_loop_stops_at_the_largest_mesh():
    # three meshes only: the bias of L = 2 stays above eps, so the loop ends
    # there with the statistical part met and no level left to add
    eps = 1e-3
    r = mlmc.estimate_adaptive(_LevelSet(3), eps, 1, 16, max_rounds=10, sampler=_model(), cost=lambda l: 8.0 ** l)
    assert r["L"] == 2 and r["err"] > eps and r["rounds"] < 11
    assert r["var_qtilde"] <= 1.2 * eps ** 2 / 2


def test_adaptive_loop_rejects_a_first_level_without_differences():
    with pytest.raises(ValueError):
        mlmc.estimate_adaptive(_LevelSet(3), 1e-3, 0, 16, sampler=_model())


# ------------------------------------------------- allocation loop (estimate)
# The pilot / eq. mlmc_num_samples / top-up loop pinned on a deterministic level
# model whose 1/N variances are known exactly: Y_l^i = m_l + a_l (-1)^i has, for
# every even count, mean m_l and 1/N variance a_l^2 (eq. sample_variance).  The
# expected sample counts below are worked out by hand from eq. mlmc_num_samples,
# not by calling the oracle's formula.

def _alternating(m, a, calls):
    def sampler(l, first, count):
        calls.append((l, first, count))
        return np.array([m[l] + a[l] * (-1.0) ** (first + i) for i in range(count)])
    return sampler


def test_estimate_allocation_on_a_known_level_model():
    # a = (0.0103, 0.0021), C = (1, 16), eps = 1e-3:
    #   sqrt(V0 C0) = 0.0103, sqrt(V1 C1) = 0.0021 * 4 = 0.0084, sum 0.0187
    #   N0 = 2e6 * 0.0103 * 0.0187 = 385.22    -> 386
    #   N1 = 2e6 * (0.0021 / 4) * 0.0187 = 19.635 -> 20
    # both even, so the variances after the top-up are unchanged and the next
    # round asks for no more samples
    calls = []
    m, a = (0.02, 1e-4), (0.0103, 0.0021)
    n, qt, vq, st = mlmc.estimate(_LevelSet(2), 1e-3, 8, max_rounds=5, sampler=_alternating(m, a, calls),
                                  cost=lambda l: (1.0, 16.0)[l])
    assert n == [386, 20]
    # pilot first on every level, then each level continues its own index range
    assert calls == [(0, 0, 8), (1, 0, 8), (0, 8, 378), (1, 8, 12)]
    assert st[0].var == pytest.approx(a[0] ** 2, rel=1e-12) and st[1].var == pytest.approx(a[1] ** 2, rel=1e-12)
    assert qt == pytest.approx(m[0] + m[1], rel=1e-12)
    # the statistical error meets eps^2 / 2 (eq. mlmc_error's variance half)
    assert vq == pytest.approx(a[0] ** 2 / 386 + a[1] ** 2 / 20, rel=1e-12)
    assert vq <= 1e-6 / 2


def test_estimate_extra_fraction_and_pilot_floor():
    # extra_fraction 0.1 scales the formula before the ceiling:
    #   385.22 * 1.1 = 423.74 -> 424;  19.635 * 1.1 = 21.60 -> 22
    calls = []
    n, _, _, _ = mlmc.estimate(_LevelSet(2), 1e-3, 8, max_rounds=5, extra_fraction=0.1,
                               sampler=_alternating((0.02, 1e-4), (0.0103, 0.0021), calls),
                               cost=lambda l: (1.0, 16.0)[l])
    assert n == [424, 22]
    # a level the formula would give fewer samples than the pilot keeps the pilot:
    #   a1 = 2e-5: N1 = 2e6 * 5e-6 * (0.0103 + 8e-5) = 0.1038 -> 1 < 8
    calls = []
    n, _, _, _ = mlmc.estimate(_LevelSet(2), 1e-3, 8, max_rounds=5,
                               sampler=_alternating((0.02, 1e-4), (0.0103, 2e-5), calls),
                               cost=lambda l: (1.0, 16.0)[l])
    # N0 = 2e6 * 0.0103 * 0.01038 = 213.83 -> 214
    assert n == [214, 8]
    assert calls == [(0, 0, 8), (1, 0, 8), (0, 8, 206)]


def test_estimate_rounds_cap_and_regrowth():
    # a level whose first 8 samples (the pilot) are quiet (+-1.3e-3) and whose
    # later ones are loud (+-2.6e-3), one level, C = 1, eps = 1.1e-5:
    #   round 1 from the pilot: N = 2 (1.3e-3)^2 / eps^2 = 27933.9 -> 27934
    #   round 2: 1/N variance of the 27934 samples (mean 0: both runs have an
    #   even count) = (8 * 1.69e-6 + 27926 * 6.76e-6) / 27934, so
    #   N = 2 V / eps^2 = 111711.5 -> 111712
    def sampler(l, first, count):
        calls.append((l, first, count))
        return np.array([(1.3e-3 if first + i < 8 else 2.6e-3) * (-1.0) ** (first + i) for i in range(count)])
    eps = 1.1e-5
    calls = []
    n, _, _, _ = mlmc.estimate(_LevelSet(1), eps, 8, max_rounds=1, sampler=sampler, cost=lambda l: 1.0)
    assert n == [27934] and calls == [(0, 0, 8), (0, 8, 27926)]
    calls = []
    n, _, _, st = mlmc.estimate(_LevelSet(1), eps, 8, max_rounds=2, sampler=sampler, cost=lambda l: 1.0)
    v1 = (8 * 1.69e-6 + 27926 * 6.76e-6) / 27934
    assert 2 * v1 / eps ** 2 == pytest.approx(111711.5, abs=0.1)
    assert n == [111712] and calls == [(0, 0, 8), (0, 8, 27926), (0, 27934, 111712 - 27934)]


def test_estimate_fixed_counts_is_plain_mlmc():
    calls = []
    n, qt, vq, st = mlmc.estimate(_LevelSet(2), 1e-3, 8, sampler=_alternating((0.02, 1e-4), (0.01, 0.002), calls),
                                  n_fixed=(10, 4))
    assert n == [10, 4] and calls == [(0, 0, 10), (1, 0, 4)]
    assert qt == pytest.approx(0.0201, rel=1e-12)


# ------------------------------------------------------- V-cycle by value
# One V-cycle z = B b is linear in b; its error propagation is
#   I - B A = S (I - P B_c P^T A) S
# with S = p(D^-1 A) the Chebyshev error polynomial of the smoother (the same
# for the zero-start pre-smoothing and the post-smoothing) and B_c the coarse
# V-cycle (the exact inverse on the one-unknown 2^3 mesh).  The dense operator
# is composed here from numpy.linalg alone and compared with the oracle's
# recursive V-cycle.

def _dense_vcycle(H, lvl, degree, lo_ratio, hi):
    A = H.As[lvl].toarray()
    if H.ns[lvl] == 2:
        return np.linalg.inv(A)
    d = np.sqrt(np.diag(A))
    Ssym = A / d[:, None] / d[None, :]
    lam, V = np.linalg.eigh(Ssym)
    p = gmg.chebyshev_polynomial(lam, degree, hi / lo_ratio, hi)
    S = (V * p) @ V.T
    S = S / d[:, None] * d[None, :]          # D^-1/2 p(D^-1/2 A D^-1/2) D^1/2 = p(D^-1 A)
    P = H.Ps[lvl].toarray()
    Bc = _dense_vcycle(H, lvl + 1, degree, lo_ratio, hi)
    I = np.eye(A.shape[0])
    E = S @ (I - P @ Bc @ P.T @ A) @ S
    return (I - E) @ np.linalg.inv(A)


@pytest.mark.parametrize("n,degree,hi", [(4, 1, 1.75), (4, 2, 1.75), (8, 1, 1.75), (8, 2, 2.0), (8, 3, 1.75)])
def test_vcycle_equals_dense_error_operator(n, degree, hi):
    kap = element_field(n, 1, seed=70 + n, spread=1.5)[0]
    H = gmg.Hierarchy(n, kap)
    Bd = _dense_vcycle(H, 0, degree, 4.0, hi)
    for s in range(3):
        b = grid_vector(n, 1, seed=80 + s)[0]
        z = H.vcycle(b, degree, 4.0, hi)
        assert np.abs(z - Bd @ b).max() <= 1e-12 * np.abs(Bd @ b).max()
    # the composed operator is symmetric (pre- and post-smoothing are adjoint)
    assert np.abs(Bd - Bd.T).max() <= 1e-10 * np.abs(Bd).max()
