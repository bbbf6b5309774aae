"""The oracle's operation counter, and the per-unit operation counts the
benchmark uses for the roofline of the cube-stack forward (bench.py
STACK_FWD_FLOPS), checked against it.

The counter (orc_flop_count) runs the oracle's own forward rollout in a
counting scalar: each add, subtract, multiply, divide, square root or
elementary function is one operation, except where an operand is a structural
zero (a literal zero of the code, such as the zero blocks of J, M and H the
dense loops visit) or a constant +-1.  It is pinned here to the closed-form
operation counts of the Cholesky factorization and triangular solves (dense,
and block diagonal, where the skipped zeros must leave exactly the per-block
count).  The per-unit table was fitted to the counter on other worlds; on the
held-out worlds below it must predict each phase within 10%.
"""
import numpy as np
import pytest

import bench
from oracle import oracle as O
from paper_2506_14186_amd import workloads as W


def _dense_count(n):
    # factorization: column j takes j products and j differences for its
    # diagonal, one square root, then (n - 1 - j) entries of j products,
    # j differences and one division; each triangular solve takes i products,
    # i differences and one division in row i
    fact = sum(2 * j + 1 + (n - 1 - j) * (2 * j + 1) for j in range(n))
    solve = 2 * sum(2 * i + 1 for i in range(n))
    return fact + solve


@pytest.mark.parametrize("n", [1, 2, 3, 6, 13])
def test_counter_dense_cholesky_closed_form(n):
    rng = np.random.default_rng(n)
    B = rng.normal(size=(n, n))
    assert O.flop_cholesky(B @ B.T + n * np.eye(n)) == _dense_count(n)


@pytest.mark.parametrize("blocks,size", [(2, 6), (5, 6), (3, 4)])
def test_counter_skips_structural_zeros(blocks, size):
    rng = np.random.default_rng(blocks * size)
    n = blocks * size
    A = np.zeros((n, n))
    for b in range(blocks):
        B = rng.normal(size=(size, size))
        A[b * size:(b + 1) * size, b * size:(b + 1) * size] = B @ B.T + size * np.eye(size)
    assert O.flop_cholesky(A) == blocks * _dense_count(size)
    # a data value that happens to be one or zero is still counted: only
    # structural zeros are skipped, so one nonzero coupling entry adds work
    A[size, 0] = A[0, size] = 0.5
    assert O.flop_cholesky(A) > blocks * _dense_count(size)


def _oracle_units(r, k):
    return {"body_attempts": r["attempts"] * k, "body_rhs": r["rhs"] * k, "pair_rhs": r["rhs"] * (k - 1),
            "rhs_contacts_plane": r["rhs_contacts"] - r["rhs_contacts_box"],
            "rhs_contacts_pair": r["rhs_contacts_box"],
            "body_newton_iters": r["newton_iters"] * k, "pair_newton_iters": r["newton_iters"] * (k - 1),
            "newton_contacts_plane": r["newton_contacts"] - r["newton_contacts_box"],
            "newton_contacts_pair": r["newton_contacts_box"]}


def _tossed(k, seed):
    rng = np.random.default_rng(seed)
    x = W.stack_state(rng.normal(0.0, 0.02, size=(k, 2)))
    for i in range(k):
        th = rng.normal(0.0, 0.15, 3)
        a = np.linalg.norm(th)
        x[7 * i + 3:7 * i + 7] = np.concatenate([[np.cos(a / 2)], np.sin(a / 2) * th / a])
        x[7 * i + 2] += 0.05 * i
    x[7 * k:] = rng.normal(0.0, 0.3, 6 * k)
    return x


def _held_out():
    cfg = W.cube_stacks(seed=9, n_worlds=64, kmax=10, horizon=0.05)
    picks = [int(w) for w in np.argsort(cfg["k"])[::9]][:6]
    out = [(cfg["models"][w], cfg["x0"][w], 0.05) for w in picks]
    out += [(W.model_stack(k, tc=0.003), _tossed(k, 20 + k), 0.03) for k in (3, 6)]
    return out


def test_stack_flop_table_predicts_oracle_counts():
    T = bench.STACK_FWD_FLOPS
    phases = {"step": ["body_attempts"],
              "rhs": ["body_rhs", "pair_rhs", "rhs_contacts_plane", "rhs_contacts_pair"],
              "newton": ["body_newton_iters", "pair_newton_iters", "newton_contacts_plane", "newton_contacts_pair"]}
    assert sorted(sum(phases.values(), [])) == sorted(T)
    worst = {p: 0.0 for p in phases}
    for desc, x, horizon in _held_out():
        k = x.size // 13
        r = O.Model(desc).flop_count(x, None, 1, horizon)
        assert r["status"] == 0
        u = _oracle_units(r, k)
        counted = {"step": r["flops_step"], "rhs": r["flops_rhs"],
                   "newton": r["flops_newton"] + r["flops_line_search"]}
        for p, names in phases.items():
            pred = sum(T[n] * u[n] for n in names)
            if counted[p] == 0:
                assert pred == 0
                continue
            dev = pred / counted[p] - 1.0
            worst[p] = max(worst[p], abs(dev))
            assert abs(dev) <= 0.10, (k, p, pred, counted[p])
    print("largest deviation of the table from the oracle's counts:", {p: round(v, 3) for p, v in worst.items()})
