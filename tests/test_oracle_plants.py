"""Planted mistakes: each plausible slip in the oracle must be caught by a pin.

Every case below rebuilds ``oracle/oracle.c`` with one small edit (a dropped
sign, a wrong index, a transposed operand ...) into a temporary library and
shows that the pins of ``test_oracle_pins.py`` reject it, while the unedited
oracle passes the same checks.  Runs on the CPU only.
"""
import os
import tempfile

import numpy as np
import pytest

import oracle
import workloads as W
from checks import orth, residual, toeplitz_121_exact, tri_dense

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

# (name, original text, planted text)
PLANTS = [
    ("z_sign_dropped", "z[n1 + i] = sg * A_(Q2", "z[n1 + i] = 1.0 * A_(Q2"),
    ("corner_once", "d[k - 1] -= rho;\n    d[k] -= rho;", "d[k - 1] -= rho;"),
    ("split_coupling_index", "double b = e[k - 1];", "double b = e[k];"),
    ("lowner_off_by_one", "for (int j = 0; j < i; ++j) w *=", "for (int j = 0; j <= i; ++j) w *="),
    ("lowner_pairing", "/ (d[j + 1] - d[i]);", "/ (d[j] - d[i] + 1e-300);"),
    ("rotation_sign", "double c = zv[j] / tau, s = -zv[p] / tau;", "double c = zv[j] / tau, s = zv[p] / tau;"),
    ("rotation_z_not_merged", "zv[j] = tau;", "zv[j] = zv[j];"),
    ("uhat_tau_sign", "return (d[i] - d[o[j]]) - tau[j];", "return (d[i] - d[o[j]]) + tau[j];"),
    ("secular_origin_flip", "if (fmid >= 0.0) {", "if (fmid < 0.0) {"),
    ("secular_missing_rho", "return 1.0 + rho * s;", "return 1.0 + s;"),
    ("update_transposed", "acc += A_(X, m, i, cs[l]) * A_(U, K, l, j);", "acc += A_(X, m, i, cs[l]) * A_(U, K, j, l);"),
    ("deflate_tol_large", "double tol = 8.0 * OR_U *", "double tol = 8.0e8 * OR_U *"),
    ("adjoint_F_sign", "acc / (lam[j] - lam[i]);", "acc / (lam[i] - lam[j]);"),
    ("adjoint_e_one_side", "ebar[a] = up + lo;", "ebar[a] = 2.0 * up;"),
    ("normalise_rho", "double r = rho * zz;", "double r = rho;"),
]


def _pins_pass(orc) -> bool:
    """A compact subset of the pins; True iff every check holds."""
    ok = True
    # whole solve: closed form (both signs of the off-diagonal), random vs LAPACK
    for off in (1.0, -1.0):
        d, e = W.toeplitz_121(100, off)
        lam, Q, _ = orc.stedc(d, e, leaf=8)
        lr, _ = toeplitz_121_exact(100, off)
        ok &= np.abs(lam - lr).max() <= 4e-13
        ok &= orth(Q) <= 1e-12 and residual(d, e, lam, Q) <= 1e-13
    d, e = W.normal(120, 3)
    lam, Q, _ = orc.stedc(d, e, leaf=8)
    wr = np.linalg.eigvalsh(tri_dense(d, e))
    ok &= np.abs(lam - wr).max() <= 1e-13 * np.abs(wr).max()
    ok &= orth(Q) <= 1e-12 and residual(d, e, lam, Q) <= 1e-13
    # merge with forced rotations and uneven halves
    D, z, rho, Q1, Q2 = W.random_merge(24, 17, seed=3, dup=5)
    lam, Q, st = orc.merge(D, z, rho, Q1, Q2)
    n1 = 24
    Qb = np.zeros((41, 41))
    Qb[:n1, :n1] = Q1
    Qb[n1:, n1:] = Q2
    A = Qb @ (np.diag(D) + rho * np.outer(z, z)) @ Qb.T
    wr = np.linalg.eigvalsh(A)
    ok &= np.abs(lam - wr).max() <= 1e-13 * np.abs(wr).max()
    ok &= orth(Q) <= 1e-12 and np.linalg.norm(A @ Q - Q * lam) / (41 * np.abs(wr).max()) <= 1e-13
    ok &= st[5] >= 5
    # adjoint vs the eigenvalue closed form and a Q-dependent finite difference
    d, e = W.ramp(12, 1)
    lam, Q, _ = orc.stedc(d, e)
    g = np.random.default_rng(0)
    wv = g.standard_normal(12)
    dbar, ebar = orc.adjoint(lam, Q, wv, np.zeros((12, 12)))
    ok &= np.allclose(dbar, (Q ** 2) @ wv, atol=1e-12) and np.allclose(ebar, 2 * (Q[:-1] * Q[1:]) @ wv, atol=1e-12)
    G = g.standard_normal((12, 12))
    dbar, ebar = orc.adjoint(lam, Q, np.zeros(12), G)
    h = 1e-6

    def L(dd, ee):
        w2, V2 = np.linalg.eigh(tri_dense(dd, ee))
        V2 = V2 * np.sign(np.sum(V2 * Q, axis=0))[None, :]
        return float(np.sum(G * V2))
    ep, em = e.copy(), e.copy()
    ep[4] += h
    em[4] -= h
    fd_e = (L(d, ep) - L(d, em)) / (2 * h)
    dp, dm = d.copy(), d.copy()
    dp[5] += h
    dm[5] -= h
    fd_d = (L(dp, e) - L(dm, e)) / (2 * h)
    ok &= abs(ebar[4] - fd_e) <= 1e-6 * max(1.0, abs(fd_e)) and abs(dbar[5] - fd_d) <= 1e-6 * max(1.0, abs(fd_d))
    return bool(ok)


def test_unplanted_oracle_passes(orc):
    assert _pins_pass(orc)


@pytest.mark.parametrize("name,orig,planted", PLANTS, ids=[p[0] for p in PLANTS])
def test_plant_is_caught(name, orig, planted):
    src = open(SRC).read()
    assert src.count(orig) == 1, f"plant site for {name} not found exactly once"
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, f"plant_{name}.c")
        with open(path, "w") as f:
            f.write(src.replace(orig, planted))
        lib = os.path.join(td, f"plant_{name}.so")
        oracle.build(src=path, out=lib)
        bad = oracle.Oracle(lib)
        try:
            caught = not _pins_pass(bad)
        except Exception:  # a crash or a non-finite result also counts as caught
            caught = True
    assert caught, f"planted mistake {name} was not caught by the pins"
