"""Pins of the oracle's chaos layer against closed forms and the paper's integers."""

import math
import os

import numpy as np
import pytest

from oracle import chaos, hsc, sg
from sg_inputs import named_problem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append([int(v) for v in line.split()])
    return rows


def hermite_triple_closed_form(a, b, c):
    """E[psi_a psi_b psi_c] for normalised probabilists' Hermite (linearisation formula)."""
    if (a + b + c) % 2:
        return 0.0
    s = (a + b + c) // 2
    if s < max(a, b, c):
        return 0.0
    f = math.factorial
    return math.sqrt(f(a) * f(b) * f(c)) / (f(s - a) * f(s - b) * f(s - c))


@pytest.mark.parametrize("M,p", [(1, 3), (2, 2), (3, 4), (4, 2), (10, 3), (8, 3)])
def test_multi_index_count_and_grading(M, p):
    al = chaos.multi_indices(M, p)
    assert al.shape == (math.comb(M + p, p), M)
    deg = al.sum(axis=1)
    assert np.all(np.diff(deg) >= 0)
    assert len({tuple(r) for r in al}) == al.shape[0]
    off = chaos.level_offsets(M, p)
    for l in range(p + 1):
        assert np.all(deg[off[l]:off[l + 1]] == l)
        assert off[l + 1] - off[l] == math.comb(M + l - 1, l)
        block = [tuple(r) for r in al[off[l]:off[l + 1]]]
        assert block == sorted(block, reverse=True)


def test_triple_products_match_linearisation_formula():
    """E[xi psi_a psi_b] = E[psi_1 psi_a psi_b] against the Hermite linearisation formula."""
    for a in range(7):
        for b in range(7):
            val = chaos.normalized_moment(1, a, b)
            assert abs(val - hermite_triple_closed_form(a, b, 1)) < 1e-13
            assert abs(val - (math.sqrt(max(a, b)) if abs(a - b) == 1 else 0.0)) < 1e-13


def test_orthonormality_by_quadrature():
    for a in range(7):
        for b in range(7):
            assert abs(chaos.normalized_moment(0, a, b) - (a == b)) < 1e-13


@pytest.mark.parametrize("M,p", [(2, 3), (4, 2), (10, 3)])
def test_galerkin_matrix_entries(M, p):
    al = chaos.multi_indices(M, p)
    Gs = chaos.galerkin_matrices(M, p)
    assert np.array_equal(Gs[0], np.eye(al.shape[0]))
    for k in range(1, M + 1):
        G = Gs[k]
        assert np.array_equal(G, G.T)
        diff = al[:, None, :] - al[None, :, :]
        only_k = (np.abs(diff).sum(axis=2) == 1) & (np.abs(diff[:, :, k - 1]) == 1)
        expect = np.where(only_k, np.sqrt(np.maximum(al[:, None, k - 1], al[None, :, k - 1])), 0.0)
        assert np.max(np.abs(G - expect)) < 1e-13
        assert np.array_equal(G != 0, only_k)


def test_block_counts_table5_and_figure1():
    for v, n_b, n_db, n_m, n_ds in _load("table5_workcounts.txt"):
        for (M, p) in [(v, 4), (4, v)]:
            pat = chaos.block_pattern(chaos.galerkin_matrices(M, p))
            assert int(np.count_nonzero(pat)) == n_b
            assert pat.shape[0] == n_db
            assert n_b - n_db == n_m
            assert 2 * (n_db - 1) + 1 == n_ds
            # closed form of the block count for a linear KL expansion
            assert math.comb(M + p, p) + 2 * M * math.comb(M + p - 1, M) == n_b
    for N, P, blocks in _load("fig1_blocks.txt"):
        pat = chaos.block_pattern(chaos.galerkin_matrices(N, P))
        assert int(np.count_nonzero(pat)) == blocks


def test_ndof_columns():
    for _tab, N, P, inv_h, ndof in _load("ndof_tables.txt"):
        assert (inv_h + 1) ** 2 * math.comb(N + P, P) == ndof


@pytest.mark.parametrize("v", [1, 2, 3])
def test_hsc_counters_match_work_counts(v):
    """Block matvecs and block solves per action of Algorithm 1 equal n_m and n_ds."""
    row = [r for r in _load("table5_workcounts.txt") if r[0] == v][0]
    for (M, p) in [(v, 4), (4, v)]:
        prob = named_problem("small", n_e=3, M=M, p=p)
        s = sg.build_system(prob)
        cnt = hsc.Counters()
        R = np.random.default_rng(0).standard_normal((s.n, s.P))
        hsc.hsc_apply(s, R, hsc.ExactMeanSolver(s), cnt)
        assert cnt.block_matvecs == row[3]
        assert cnt.block_solves == row[4]
