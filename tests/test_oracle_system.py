"""Pins of the oracle's pair precompute, Alg. 3 matvec, GMRES and post-processing.

* P4  isolated pair: Alg. 3 collapses to T = I exactly, whatever A is (Sec. 3.5:
      the two-body system of an isolated pair is designed to be the identity).
* P5  brute force on tiny inputs: the compressed method against a direct
      fine-grid MFS solve of the same 2- and 3-body problems (no compression,
      no preconditioning).  With the paper's coarse parameters (N_c = 60,
      M_c = 72, R_c = 1 - ln(1e12)/60) the two agree to MFS accuracy.
* P6  dense T assembled column by column from Alg. 3 equals T assembled from
      the closed masked formula; GMRES agrees with a dense LU solve.
* P7  exact symmetries of the discrete system: rotation by pi about any point,
      reflection y -> -y and translation map every point set onto itself.
* P8  two-way consistency (Sec. 6.1): resistance output fed to mobility
      returns the input; reciprocity of the mobility matrix.
* P10 peanut compression: the coarse sources reproduce the fine correction
      field outside the peanut.
"""

import math

import numpy as np
import pytest

from oracle.direct import direct_solve
from oracle.geometry import fine_nodes, fine_sources, ring, ring_radius
from oracle.kernel import direct_sum
from oracle.pairs import pair_matrices
from oracle.params import MFSParams
from oracle.system import System, gmres, rel_rigid_error, solve

PAPER_COARSE = (60, 72, 1 - 12 * math.log(10) / 60)   # Sec. 6.2 run: N_c = 60, 72 nodes, ring rule
SMALL = MFSParams(n_fp=60, n_ell=30, m_p=100)            # cheap fine grids for bookkeeping tests


def _pair(delta, ang=0.7, c0=(0.1, 0.2)):
    c0 = np.array(c0)
    return np.array([c0, c0 + (2 + delta) * np.array([math.cos(ang), math.sin(ang)])])


@pytest.mark.parametrize("problem", ["mobility", "resistance"])
def test_isolated_pair_is_identity(problem):
    for delta in (1e-3, 0.05):
        S = System(_pair(delta), 1.0, 36, 72, 0.7, problem, SMALL)
        v = np.random.default_rng(0).standard_normal(S.n)
        assert np.max(np.abs(S.matvec(v) - v)) < 1e-10 * np.max(np.abs(v))
        assert np.max(np.abs(S.matvec_masked(v) - v)) == 0.0
        assert np.max(np.abs(S.matvec_W(v) - v)) < 1e-6 * np.max(np.abs(v))


def _fine_ring_body(c, prm):
    Rf = ring_radius(prm.n_fp, prm.eps_ring)
    return (c, ring(c, Rf, prm.n_fp), ring(c, 1.0, int(math.ceil(prm.a_f * prm.n_fp))))


@pytest.mark.parametrize("problem", ["mobility", "resistance"])
def test_brute_force_pair_and_triple(problem):
    prm = MFSParams()
    rng = np.random.default_rng(5)
    nc, mc, rc = PAPER_COARSE
    c = np.array([[0.0, 0.0], [2.001, 0.0], [1.0, 2.6]])
    for P in (2, 3):
        g = rng.standard_normal((P, 3))
        if problem == "mobility":
            g[:, :2] -= g[:, :2].mean(0)
        S = System(c[:P], 1.0, nc, mc, rc, problem, prm)
        out, _, info = solve(S, g, 1e-13)
        Yi, Yk = fine_sources(c[0], c[1], prm)
        Xi, Xk = fine_nodes(c[0], c[1], prm)
        bodies = [(c[0], Yi, Xi), (c[1], Yk, Xk)] + ([_fine_ring_body(c[2], prm)] if P == 3 else [])
        ref = direct_solve(bodies, g, problem)
        err = rel_rigid_error(out, ref).max()
        assert err < 2e-6, (problem, P, err)
        if P == 3:
            # the pair correction A matters: dropping it (one-body coupling only) is far off
            for d in S.pd:
                d["A"] = np.zeros_like(d["A"])
            out0, _, _ = solve(S, g, 1e-13)
            assert rel_rigid_error(out0, ref).max() > 100 * err


def _cluster4():
    # a chain of two contacts plus a third contact: pairs (0,1), (1,2), (2,3) and a far-ish body
    return np.array([[0.0, 0.0], [2.01, 0.0], [3.0, 1.75], [5.0, 1.9]])


@pytest.mark.parametrize("problem", ["mobility", "resistance"])
def test_dense_alg3_equals_masked_form_and_lu(problem):
    c = _cluster4()
    S = System(c, 1.0, 12, 24, 0.7, problem, MFSParams(n_fp=40, n_ell=20, m_p=60, delta_c=0.3))
    assert len(S.pairs) >= 3
    T1 = S.dense()
    T2 = S.dense(masked=True)
    assert np.max(np.abs(T1 - T2)) < 1e-9 * np.max(np.abs(T1))
    g = np.random.default_rng(1).standard_normal((4, 3))
    b = S.rhs(g)
    x_lu = np.linalg.solve(T2, b)
    x_gm, info = gmres(S.matvec, b, 1e-13)
    assert np.linalg.norm(x_gm - x_lu) < 1e-10 * np.linalg.norm(x_lu)
    assert info["true_resid"] < 1e-12


def _transform(c, g, kind):
    if kind == "rot":      # rotation by pi about (0.3, -0.2): v -> -v, omega -> omega
        return 2 * np.array([0.3, -0.2]) - c, g * np.array([-1, -1, 1])
    if kind == "refl":     # reflection y -> -y: (vx, vy, omega) -> (vx, -vy, -omega)
        return c * np.array([1, -1]), g * np.array([1, -1, -1])
    if kind == "shift":
        return c + np.array([17.25, -3.5]), g
    raise ValueError(kind)


@pytest.mark.parametrize("problem", ["mobility", "resistance"])
@pytest.mark.parametrize("kind", ["rot", "refl", "shift"])
def test_exact_symmetries(problem, kind):
    c = np.array([[0.0, 0.0], [2.003, 0.1], [1.2, 2.05], [-2.3, 0.4]])
    g = np.random.default_rng(2).standard_normal((4, 3))
    if problem == "mobility":
        g[:, :2] -= g[:, :2].mean(0)
    S = System(c, 1.0, 36, 72, 0.7, problem, SMALL)
    out, _, _ = solve(S, g, 1e-13)
    c2, g2 = _transform(c, g, kind)
    S2 = System(c2, 1.0, 36, 72, 0.7, problem, SMALL)
    out2, _, _ = solve(S2, g2, 1e-13)
    _, back = _transform(np.zeros((4, 2)), out2, kind)
    assert rel_rigid_error(back, out).max() < 1e-8   # rounding, amplified by the 1e-11 fine truncation


def test_two_way_and_reciprocity():
    nc, mc, rc = PAPER_COARSE
    prm = MFSParams()
    # Two-way error (Sec. 6.1): both problems fix w = 0 (Remark 1), so mobility inverts
    # resistance; the round trip error is the MFS error amplified by the conditioning
    # of the resistance matrix, so use a moderate gap here.
    c = np.array([[0.0, 0.0], [2.05, 0.0], [1.0, 2.3]])
    R = System(c, 1.0, nc, mc, rc, "resistance", prm)
    M = System(c, 1.0, nc, mc, rc, "mobility", prm)
    vw = np.random.default_rng(3).standard_normal((3, 3))
    ft, _, _ = solve(R, vw, 1e-13)
    back, _, _ = solve(M, ft, 1e-13)
    assert rel_rigid_error(back, vw).max() < 1e-6
    c = np.array([[0.0, 0.0], [2.002, 0.0], [1.0, 2.3]])
    M = System(c, 1.0, nc, mc, rc, "mobility", prm)
    # mobility matrix from unit solves is symmetric to MFS accuracy
    Mm = np.zeros((9, 9))
    for j in range(9):
        e = np.zeros(9)
        e[j] = 1.0
        Mm[:, j] = solve(M, e.reshape(3, 3), 1e-13)[0].reshape(-1)
    assert np.max(np.abs(Mm - Mm.T)) < 1e-5 * np.max(np.abs(Mm))


def test_peanut_compression_reproduces_far_field():
    prm = MFSParams()
    for problem in ("mobility", "resistance"):
        from oracle.onebody import one_body
        ob = one_body(1.0, 36, 72, 0.7, 1.0, problem, 1e-14)
        c = _pair(1e-3)
        d = pair_matrices(c[0], c[1], ob, prm, keep=True)
        x = np.random.default_rng(4).standard_normal(d["A"].shape[1])
        beta = -(d["G"] @ x)
        lt = d["A"] @ x
        if problem == "mobility":
            from scipy.linalg import block_diag
            from oracle.geometry import rigid_projector
            Kfi, Kfk = d["Kfi"], d["Kfk"]
            beta = block_diag(np.eye(Kfi.shape[0]) - rigid_projector(Kfi),
                              np.eye(Kfk.shape[0]) - rigid_projector(Kfk)) @ beta
            lt = block_diag(ob.IL, ob.IL) @ lt
        Yc = np.concatenate([c[0] + ob.Yr, c[1] + ob.Yr])
        # evaluation points outside the peanut: at distance >= 1.3 from both centres... on a far circle
        t = np.linspace(0, 2 * math.pi, 50, endpoint=False)
        mid = c.mean(0)
        pts = mid + 3.0 * np.stack([np.cos(t), np.sin(t)], axis=1)
        uf = direct_sum(pts, d["Yf"], beta.reshape(-1, 2))
        uc = direct_sum(pts, Yc, lt.reshape(-1, 2))
        assert np.max(np.abs(uf - uc)) < 1e-7 * np.max(np.abs(uf))


# -- unequal radii (the bidisperse workload; a reading of the paper) ---------------------------------------

def _unequal_pair(delta, a=(1.0, 1.4), ang=0.7, c0=(0.1, 0.2)):
    c0 = np.array(c0)
    return np.array([c0, c0 + (a[0] + a[1] + delta) * np.array([math.cos(ang), math.sin(ang)])]), np.array(a)


@pytest.mark.parametrize("problem", ["mobility", "resistance"])
def test_isolated_unequal_pair_is_identity(problem):
    # P4 for radii 1 and 1.4 (36/72 and 50/100 coarse points): T = I whatever A is.  The
    # closed masked form gives I exactly; the literal Alg. 3 adds and cancels terms carrying
    # lambda_bar, which the one-body pseudoinverse of the 50-source disk amplifies ~100x more
    # than the 36-source one's (1e-10 for unit pairs), so it is held to 1e-8.
    for delta in (1e-3, 0.05):
        c, a = _unequal_pair(delta)
        S = System(c, a, [36, 50], [72, 100], 0.7, problem, SMALL)
        assert S.pd[0]["A"].shape == (2 * (36 + 50), 2 * (36 + 50))
        v = np.random.default_rng(1).standard_normal(S.n)
        assert np.max(np.abs(S.matvec(v) - v)) < 1e-8 * np.max(np.abs(v))
        assert np.max(np.abs(S.matvec_masked(v) - v)) == 0.0


@pytest.mark.parametrize("problem", ["mobility", "resistance"])
def test_brute_force_unequal_pair(problem):
    # P5 for radii 1 and 1.4 at gap 1e-3: the compressed method against a direct fine-grid
    # solve on the pair's own fine sets.  Coarse sizes scale with the radius (paper's 60/72
    # at radius 1, 84/100 at 1.4, ring rule for the source radius).
    prm = MFSParams()
    c, a = _unequal_pair(1e-3)
    ns = [60, 84]
    nc = [72, 100]
    rs = [1 - 12 * math.log(10) / n for n in ns]
    g = np.random.default_rng(6).standard_normal((2, 3))
    if problem == "mobility":
        g[:, :2] -= g[:, :2].mean(0)
    S = System(c, a, ns, nc, rs, problem, prm)
    out, _, _ = solve(S, g, 1e-13)
    Yi, Yk = fine_sources(c[0], c[1], prm, a[0], a[1])
    Xi, Xk = fine_nodes(c[0], c[1], prm, a[0], a[1])
    ref = direct_solve([(c[0], Yi, Xi), (c[1], Yk, Xk)], g, problem)
    err = rel_rigid_error(out, ref).max()
    assert err < 2e-6, (problem, err)
