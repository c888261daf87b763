"""CPU oracle of the energy test -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU baseline may
use this module.  It shares no code with the HIP path.

Follows the paper's Sect. 2.2 (energy test) and Sect. 3 (background) directly:

* coordinates: invariant masses of particle combinations (Sect. 4.2, Table 1),
  computed from the stored four-vectors in float64; for D0 -> pi+ pi- pi+ pi-
  the pions are first labelled by the rule of Sect. 4.2 (the pi+ pi- pair of
  largest invariant mass is pi3 pi4), see ``d4pi_perm``;
* psi_ij = exp(-d_ij^2 / (2 sigma^2)), d_ij the Euclidean distance between the
  coordinate vectors of events i and j (Sect. 2.2);
* T of eq. (2): the two within-sample averages over pairs i < j minus the
  cross-sample average over all pairs;
* T of eq. (3): the same with the background-sample terms, written as double
  sums over ordered pairs (j != i within a sample) with the paper's factors;
* permutation p-value: the fraction of permutation T values above the observed
  one (Sect. 2.2).

All sums are plain float64 over explicit pairs (blocked only to bound memory).
"""
from __future__ import annotations

import os
from fractions import Fraction

import numpy as np


# the four pi+ pi- pairs of (+ - + -) slots, and the labelling that makes each
# of them pi3 pi4 (new slot t holds stored slot perm[t]); listed in the order
# that decides ties: the stored labelling, then both pairs swapped, then the
# pi+ swapped, then the pi- swapped
D4PI_PAIRS = ((2, 3), (0, 1), (0, 3), (2, 1))
D4PI_PERMS = ((0, 1, 2, 3), (2, 3, 0, 1), (2, 1, 0, 3), (0, 3, 2, 1))


def _pair_m2(x, a, b):
    S = x[a] + x[b]
    return S[0] ** 2 - S[1] ** 2 - S[2] ** 2 - S[3] ** 2


def _pair_m2_exact(x, i, a, b):
    S = [Fraction(float(x[a][c][i])) + Fraction(float(x[b][c][i])) for c in range(4)]
    return S[0] ** 2 - S[1] ** 2 - S[2] ** 2 - S[3] ** 2


def d4pi_perm(comps):
    """Per event, the index (into D4PI_PERMS) of the labelling of Sect. 4.2 for
    D0 -> pi+ pi- pi+ pi- stored in charge order: the pi+ pi- pair with the
    largest invariant mass becomes pi3 pi4.  Masses squared in float64; a
    comparison within 1e-9 of the pair's magnitude scale is redone in exact
    rational arithmetic; equal masses keep the earlier pair of D4PI_PAIRS."""
    x = np.asarray(comps, dtype=np.float64)
    n = x.shape[2]
    m2 = np.array([_pair_m2(x, a, b) for a, b in D4PI_PAIRS])
    scale = np.array([(np.abs(x[a]) + np.abs(x[b])).sum(axis=0) ** 2 for a, b in D4PI_PAIRS])
    best = np.zeros(n, dtype=np.int64)
    idx = np.arange(n)
    for k in range(1, 4):
        d = m2[k] - m2[best, idx]
        near = np.abs(d) <= 1e-9 * (scale[k] + scale[best, idx])
        best = np.where(~near & (d > 0), k, best)
        for i in np.nonzero(near)[0]:
            a, b = D4PI_PAIRS[k]
            c, e = D4PI_PAIRS[best[i]]
            if _pair_m2_exact(x, i, a, b) > _pair_m2_exact(x, i, c, e):
                best[i] = k
    return best


def invariant_masses(comps, masks, relabel=None):
    """Invariant mass of the slots in each bit mask, per event.

    comps: [4 slots][4 comps (E, px, py, pz)][n]; masks: iterable of slot bit
    masks.  Returns float64 [len(masks)][n]; m = sqrt(max(m^2, 0)).
    relabel="d4pi": slots hold pi+ pi- pi+ pi- and are labelled by ``d4pi_perm``
    before the masses are formed.
    """
    x = np.asarray(comps, dtype=np.float64)
    if relabel == "d4pi":
        best = d4pi_perm(x)
        perm = np.array(D4PI_PERMS)[best]          # [n][4]
        idx = np.arange(x.shape[2])
        x = np.stack([x[perm[:, t], :, idx].T for t in range(4)])
    elif relabel is not None:
        raise ValueError("relabel must be None or 'd4pi'")
    out = []
    for m in masks:
        S = np.zeros((4, x.shape[2]))
        for s in range(4):
            if m & (1 << s):
                S += x[s]
        m2 = S[0] ** 2 - S[1] ** 2 - S[2] ** 2 - S[3] ** 2
        out.append(np.sqrt(np.maximum(m2, 0.0)))
    return np.array(out)


def psi_block(Ya, Yb, sigma):
    """psi for every pair of a block: Ya [D][na], Yb [D][nb] -> [na][nb]."""
    d2 = np.zeros((Ya.shape[1], Yb.shape[1]))
    for k in range(Ya.shape[0]):
        diff = Ya[k][:, None] - Yb[k][None, :]
        d2 += diff * diff
    return np.exp(-d2 / (2.0 * sigma * sigma))


def pair_sum(Ya, Yb, sigma, same, block=2048):
    """sum of psi over pairs: same sample (Ya is Yb): ordered pairs with j != i;
    different samples: all pairs (i in a, j in b)."""
    Ya = np.asarray(Ya, dtype=np.float64)
    Yb = np.asarray(Yb, dtype=np.float64)
    na, nb = Ya.shape[1], Yb.shape[1]
    tot = 0.0
    for i0 in range(0, na, block):
        for j0 in range(0, nb, block):
            p = psi_block(Ya[:, i0:i0 + block], Yb[:, j0:j0 + block], sigma)
            if same and i0 == j0:
                np.fill_diagonal(p, 0.0)
            tot += float(p.sum())
    return tot


def column_pair_sums(Y, G, sigma, block=2048):
    """M[c][d] = sum over ordered pairs i != j of G[i][c] psi_ij G[j][d] for 0/1 (or
    any real) columns G [n][C]: each pair sum of eq. (2) / eq. (3) between two event
    sets is one entry (S(A, B) = M[a][b] for disjoint sets a, b; S(A, A) over
    ordered pairs = M[a][a]).  psi is formed block by block in float64 and
    contracted with the columns, so many splits of the same events cost one pass
    over the pairs."""
    Y = np.asarray(Y, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    n = Y.shape[1]

    def rows(i0):                       # one block of rows against every column block
        M = np.zeros((G.shape[1], G.shape[1]))
        for j0 in range(0, n, block):
            p = psi_block(Y[:, i0:i0 + block], Y[:, j0:j0 + block], sigma)
            if i0 == j0:
                np.fill_diagonal(p, 0.0)
            M += G[i0:i0 + block].T @ (p @ G[j0:j0 + block])
        return M

    # row blocks on the host's cores (numpy releases the interpreter lock)
    from concurrent.futures import ThreadPoolExecutor
    workers = min(16, os.cpu_count() or 1, max(1, (n + block - 1) // block))
    with ThreadPoolExecutor(workers) as ex:
        return sum(ex.map(rows, range(0, n, block)))


def T_eq2_columns(M, a, b, n, nb):
    """eq. (2) from column pair sums: sets a (n events) and b (nb events) are
    columns of ``column_pair_sums``; within-sample sums over pairs i < j are
    half the ordered-pair sums."""
    return 0.5 * M[a][a] / (n * (n - 1)) + 0.5 * M[b][b] / (nb * (nb - 1)) - M[a][b] / (n * nb)


def T_eq3_columns(M, A, Ab, Bk, Bkb, n, nb, bs, bsb, b, b_bar, terms=False):
    """eq. (3) from column pair sums: columns A, Ab (main samples, n and nb events),
    Bk, Bkb (background samples, bs and bsb events) of ``column_pair_sums``.  With
    ``terms`` the ten coefficient x pair-sum terms are returned as three lists
    (T = sum(t1) + sum(t2) - sum(t3) after the division by each bracket's
    normalisation, which is applied to the returned terms)."""
    w, wb = n - b, nb - b_bar
    t1 = [M[A][A], -2.0 * b / bs * M[A][Bk], b * (b + 1.0) / (bs * (bs - 1.0)) * M[Bk][Bk]]
    t2 = [M[Ab][Ab], -2.0 * b_bar / bsb * M[Ab][Bkb], b_bar * (b_bar + 1.0) / (bsb * (bsb - 1.0)) * M[Bkb][Bkb]]
    t3 = [M[A][Ab], -b_bar / bsb * M[A][Bkb], -b / bs * M[Bk][Ab], b * b_bar / (bs * bsb) * M[Bk][Bkb]]
    t1 = [t / (2.0 * w * (w - 1.0)) for t in t1]
    t2 = [t / (2.0 * wb * (wb - 1.0)) for t in t2]
    t3 = [t / (w * wb) for t in t3]
    if terms:
        return t1, t2, t3
    return sum(t1) + sum(t2) - sum(t3)


def T_eq2(Y, label, sigma):
    """eq. (2): samples are the events with label 1 (n of them) and label 0
    (nbar).  Within-sample sums run over pairs i < j."""
    Y = np.asarray(Y, dtype=np.float64)
    label = np.asarray(label).astype(bool)
    X, Xb = Y[:, label], Y[:, ~label]
    n, nb = X.shape[1], Xb.shape[1]
    s_xx = 0.5 * pair_sum(X, X, sigma, True)          # pairs i < j
    s_bb = 0.5 * pair_sum(Xb, Xb, sigma, True)
    s_xb = pair_sum(X, Xb, sigma, False)
    return s_xx / (n * (n - 1)) + s_bb / (nb * (nb - 1)) - s_xb / (n * nb)


def T_eq3(main, main_bar, bkg, bkg_bar, b, b_bar, sigma):
    """eq. (3): main samples (n, nbar events) contain b and b_bar background
    events; background samples hold b_s and b_s_bar events.  w = n - b signal
    events (w_bar likewise).  Within-sample double sums run over j != i."""
    n, nb = main.shape[1], main_bar.shape[1]
    bs, bsb = bkg.shape[1], bkg_bar.shape[1]
    w, wb = n - b, nb - b_bar
    S = lambda A, B, same=False: pair_sum(A, B, sigma, same)
    t1 = (S(main, main, True) - 2.0 * b / bs * S(main, bkg)
          + b * (b + 1.0) / (bs * (bs - 1.0)) * S(bkg, bkg, True)) / (2.0 * w * (w - 1.0))
    t2 = (S(main_bar, main_bar, True) - 2.0 * b_bar / bsb * S(main_bar, bkg_bar)
          + b_bar * (b_bar + 1.0) / (bsb * (bsb - 1.0)) * S(bkg_bar, bkg_bar, True)) / (2.0 * wb * (wb - 1.0))
    t3 = (S(main, main_bar) - b_bar / bsb * S(main, bkg_bar) - b / bs * S(bkg, main_bar)
          + b * b_bar / (bs * bsb) * S(bkg, bkg_bar)) / (w * wb)
    return t1 + t2 - t3


def p_value(T_obs, T_perm):
    """Fraction of permutation T values greater than the observed one."""
    T_perm = np.asarray(T_perm, dtype=np.float64)
    return float(np.count_nonzero(T_perm > T_obs)) / len(T_perm)
