"""The error bounds behind the stop rule's row weights and the PR_VERIFY check, pinned
against exact solutions on small graphs.  No GPU: the formulas are evaluated in numpy
from their definitions and compared with dense solves (oracle.dense, numpy.linalg).

* F_j = ||(I - cP)^{-1} e_j||_1 with P's dangling columns zero (Eq. 4, dangling
  vertices absorbing): F_j = 1 at a dangling j and F_j = 1 + c delta_j + (c / deg j)
  sum_{k in out_N(j)} F_k otherwise; iterating from 1 / (1 - c) gives upper bounds
  that decrease to F.
* Folded IFP2 (Algorithm 3, phase 2 on the final pibar + h): the unnormalised error
  is sum_N g_i h_i exactly, g_i = F_i - 1 - c delta_i.
* For any pi > 0 and any beta > 0, with r_beta = beta p - (I - cP) pi:
  ||pi - pi*||_1 <= 2 sum_j F_j |r_beta,j| / sum(pi) + |sum(pi) - 1|; the library
  tries beta = b = c d^T pi + (1 - c) sum(pi) (r_b = P'' pi - pi) and beta = the ratio
  pi_j / p_j over the vertices without in-edges, for which an IFP output's bound
  equals the stop rule's 2 sum_N g_i h_i / S_x.  Also
  ||pi - pi*||_1 <= ||r_b||_1 / (1 - c) + |sum(pi) - 1| (P'' contracts by c).
"""
import numpy as np
import pytest

import oracle
import prgen

C = 0.85

GRAPHS = [
    prgen.random_digraph(60, 300, seed=11, dangling_frac=0.2, unref_frac=0.1),
    prgen.random_digraph(40, 200, seed=12, self_loops=True, multi=True, dangling_frac=0.3),
    prgen.workload_dag(n_layers=6, layer_size=12, zmax=8, target_edges=150, back_frac=0.05, seed=5),
]


def _dense(g):
    n = g.n
    deg = np.diff(g.row_ptr)
    P = np.zeros((n, n))
    for j in range(n):
        for e in range(g.row_ptr[j], g.row_ptr[j + 1]):
            P[g.col[e], j] += 1.0 / deg[j]
    nd = deg > 0
    ndn = np.zeros(n)
    for j in range(n):
        for e in range(g.row_ptr[j], g.row_ptr[j + 1]):
            ndn[j] += 1.0 if nd[g.col[e]] else 0.0
    delta = np.where(nd, 1.0 - ndn / np.maximum(deg, 1), 0.0)
    return P, deg, nd, delta


def _weights_iterated(g, c, iters):
    P, deg, nd, delta = _dense(g)
    f = np.where(nd, 1.0 / (1.0 - c), 1.0)
    out = [f]
    for _ in range(iters):
        # (c / deg j) sum over j's out-neighbours k in N of f_k = c * (P^T restricted to N targets) f
        acc = (P * nd[:, None]).T @ f
        f = np.where(nd, 1.0 + c * delta + c * acc, 1.0)
        out.append(f)
    return out


def _beta2(g, pi, p):
    """pi_j / p_j summed over the vertices without in-edges (None if they carry no p)."""
    noin = np.bincount(np.asarray(g.col, dtype=np.int64), minlength=g.n) == 0
    ps = p[noin].sum()
    return pi[noin].sum() / ps if ps > 0 else None


def _bounds(g, c, pi, p, F, beta=None):
    """(weighted bound at beta (default b), contraction bound)."""
    P, deg, _, _ = _dense(g)
    b = c * pi[deg == 0].sum() + (1 - c) * pi.sum()
    r = np.abs(c * (P @ pi) + b * p - pi)
    rb = r if beta is None else np.abs(c * (P @ pi) + beta * p - pi)
    tail = abs(pi.sum() - 1.0)
    return 2.0 * float((F * rb).sum()) / pi.sum() + tail, r.sum() / (1 - c) + tail


@pytest.mark.parametrize("gi", range(len(GRAPHS)))
def test_absorbing_weights(gi):
    g = GRAPHS[gi]
    P, _, nd, _ = _dense(g)
    F = np.linalg.inv(np.eye(g.n) - C * P).sum(axis=0)
    it = _weights_iterated(g, C, 40)
    assert np.allclose(it[-1], F, rtol=1e-6)
    assert F.max() <= 1.0 / (1.0 - C) + 1e-12 and np.all(F[~nd] == 1.0)
    for a, b in zip(it, it[1:]):
        assert np.all(b <= a + 1e-15) and np.all(b >= F - 1e-12)  # decreasing upper bounds


@pytest.mark.parametrize("gi", range(len(GRAPHS)))
@pytest.mark.parametrize("passes", [1, 3, 6])
def test_folded_error_equals_weighted_residual(gi, passes):
    g = GRAPHS[gi]
    P, deg, nd, delta = _dense(g)
    F = np.linalg.inv(np.eye(g.n) - C * P).sum(axis=0)
    r = oracle.ifp2(g, C, xi=1e-300, max_passes=passes)
    h0 = np.ones(g.n)
    y = np.linalg.solve(np.eye(g.n) - C * P, h0)  # exact unnormalised vector
    z = np.zeros(g.n)
    z[nd] = r["pibar"][nd] + r["h"][nd]
    z[~nd] = h0[~nd] + C * (P @ z)[~nd]  # phase 2 from the folded non-dangling values
    err = y - z
    gw = np.where(nd, F - 1.0 - C * delta, 0.0)
    assert np.all(err >= -1e-12)
    assert abs(err.sum() - float((gw * r["h"]).sum())) <= 1e-10 * max(1.0, err.sum())
    # the uniform factor c / (1 - c) bounds the same error, less tightly
    assert err.sum() <= C / (1 - C) * r["h"][nd].sum() + 1e-12


def _perturbations(g, y, rng):
    """Normalised vectors near y / |y|: random relative noise, a uniform scale, and
    y +- eps (I - cP)^{-1} e_k for every vertex k (the residual then sits on one row)."""
    P, _, _, _ = _dense(g)
    R = np.linalg.inv(np.eye(g.n) - C * P)
    star = y / y.sum()
    out = [np.abs(star * (1 + 1e-3 * rng.standard_normal(g.n))), star * 1.001]
    for k in range(g.n):
        for sgn in (1.0, -1.0):
            u = y + sgn * 1e-3 * y[k] * R[:, k]
            if u.min() > 0:
                out.append(u / u.sum())
    return out


@pytest.mark.parametrize("gi", range(len(GRAPHS)))
@pytest.mark.parametrize("passes", [2, 5])
def test_second_scale_recovers_the_stop_rule(gi, passes):
    """On a folded IFP2 output (oracle state after some passes, normalised), the weighted
    bound at beta = pi_j / p_j over the vertices without in-edges is exactly the stop
    rule's 2 sum_N g_i h_i / S_x (at beta = b it differs either way, so the check takes
    the smaller of the two)."""
    g = GRAPHS[gi]
    P, deg, nd, delta = _dense(g)
    F = np.linalg.inv(np.eye(g.n) - C * P).sum(axis=0)
    if not np.any(np.bincount(g.col, minlength=g.n) == 0):
        pytest.skip("every vertex has an in-edge")
    r = oracle.ifp2(g, C, xi=1e-300, max_passes=passes)
    h0 = np.ones(g.n)
    z = np.zeros(g.n)
    z[nd] = r["pibar"][nd] + r["h"][nd]
    z[~nd] = h0[~nd] + C * (P @ z)[~nd]
    pi = z / z.sum()
    p = np.full(g.n, 1.0 / g.n)
    gw = np.where(nd, F - 1.0 - C * delta, 0.0)
    stop = 2.0 * float((gw * r["h"]).sum()) / z.sum()
    w2, _ = _bounds(g, C, pi, p, F, _beta2(g, pi, p))
    assert abs(w2 - stop) <= 1e-9 * max(stop, 1e-300) + 1e-15, (w2, stop)


@pytest.mark.parametrize("gi", range(len(GRAPHS)))
def test_verify_bounds_hold(gi):
    g = GRAPHS[gi]
    _, _, nd, _ = _dense(g)
    F = _weights_iterated(g, C, 16)[-1]
    rng = np.random.default_rng(gi)
    for ppr in (False, True):
        p = np.full(g.n, 1.0 / g.n)
        if ppr:
            p = np.zeros(g.n)
            p[int(np.flatnonzero(nd)[0])] = 1.0
        star = oracle.dense(g, C, p)
        y = star / (C * star[~nd].sum() + (1 - C))  # (I - cP) y = p
        for pi in _perturbations(g, y, rng):
            d = np.abs(pi - star).sum()
            w, plain = _bounds(g, C, pi, p, F)
            assert d <= w * (1 + 1e-9) and d <= plain * (1 + 1e-9), (ppr, d, w, plain)
            for beta in (_beta2(g, pi, p), 0.5 * pi.sum(), 3.0):  # any positive scale
                if beta:
                    w2, _ = _bounds(g, C, pi, p, F, beta)
                    assert d <= w2 * (1 + 1e-9), (ppr, beta, d, w2)


def test_verify_weighted_bound_needs_its_factor_two():
    """On the layered DAG some perturbation's error exceeds half the weighted bound, so
    the normalisation factor 2 cannot be dropped."""
    g = GRAPHS[2]
    _, _, nd, _ = _dense(g)
    F = _weights_iterated(g, C, 16)[-1]
    p = np.full(g.n, 1.0 / g.n)
    star = oracle.dense(g, C, p)
    y = star / (C * star[~nd].sum() + (1 - C))
    worst = 0.0
    for pi in _perturbations(g, y, np.random.default_rng(0)):
        if abs(pi.sum() - 1.0) > 1e-12:
            continue  # the scaled vector: its error is the sum term alone
        w, _ = _bounds(g, C, pi, p, F)
        worst = max(worst, np.abs(pi - star).sum() / w)
    assert 0.5 < worst <= 1.0 + 1e-9, worst


@pytest.mark.parametrize("gi", range(len(GRAPHS)))
@pytest.mark.parametrize("groups", [2, 3, 5])
@pytest.mark.parametrize("unit", [False, True])
def test_ordered_sweep_residual_bookkeeping(gi, groups, unit):
    """An ordered sweep (vertex groups as id ranges, each reserving then pushing along its
    non-dangling out-edges before the next group reserves) leaves sum_N g_i h_i equal to
    the groups' residual left behind at their reserve plus c times the pushed mass weighted
    by qle_u = (1 / deg u) sum of g over u's non-dangling out-neighbours in u's group or an
    earlier one: the sums the library's ordered sweeps keep instead of a summing pass (with
    the stop rule's weights for single solves; with unit weights, S_N itself, for batched
    solves)."""
    g = GRAPHS[gi]
    n = g.n
    deg = np.diff(g.row_ptr)
    nd = deg > 0
    rng = np.random.default_rng(7 + gi)
    w = rng.random(n) + 0.1          # any positive weights: the identity is linear in them
    if unit:
        w = np.ones(n)
    h = rng.random(n) * 3.0
    xi = 1.0
    ends = [int(round(n * (q + 1) / groups)) for q in range(groups)]
    group = np.searchsorted(np.array(ends), np.arange(n), side="right")
    inact, pushed = 0.0, 0.0
    for q in range(groups):
        lo, hi = (ends[q - 1] if q else 0), ends[q]
        taken = []
        for i in range(lo, hi):
            if not nd[i]:
                continue
            if h[i] > xi:
                taken.append((i, h[i]))
                h[i] = 0.0
            else:
                inact += w[i] * h[i]
        for u, v in taken:
            qle = 0.0
            for e in range(g.row_ptr[u], g.row_ptr[u + 1]):
                j = g.col[e]
                if nd[j]:
                    h[j] += C * v / deg[u]
                    if group[j] <= group[u]:
                        qle += w[j]
            pushed += v * qle / deg[u]
    direct = float((w[nd] * h[nd]).sum())
    assert abs(direct - (inact + C * pushed)) <= 1e-12 * max(1.0, direct), (direct, inact + C * pushed)
