"""Pins of the oracle's GMRES, (O)RAS preconditioner, adjoint and IMEX step (CPU only).

Independent facts used: dense LU solutions; GMRES with restart >= n
terminating in at most n steps; the ILU(0) defining identity (LU)_ik = a_ik on
the pattern and its equality with exact LU when there is no fill; RAS
partition of unity and disjoint ownership; one subdomain with exact local
solves is A^-1 (one iteration); alpha -> infinity turns ORAS into RAS;
the preconditioner does not change the solution; the loss is quadratic in f,
so central differences are exact; a spatially uniform Gray-Scott state
follows the explicit-Euler reaction ODE exactly because A 1 = c 1.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import adjoint, krylov, reaction, schwarz, surfaces
from oracle import band as OB
from paper_2110_06322_amd import inputs
from tests import oracle_cases as C


def test_gmres_matches_dense_solve_circle_h005():
    bd, E, Om, A, P = C.circle_h005()
    f = 2.0 * inputs.circle_sin(bd.cp_active)
    x, info = krylov.fgmres(A, f, restart=30, rtol=1e-10)
    xd = np.linalg.solve(A.toarray(), f)
    assert info["converged"] and info["relres"] <= 1e-10
    assert np.abs(x - xd).max() / np.abs(xd).max() < 1e-9


def test_gmres_full_restart_terminates_in_n_steps():
    bd, E, Om, A, P = C.matrices("circle", (1.0,), 2, 0.2, 2, 1.0)
    n = bd.n_active
    f = inputs.normal(5, 0, bd.active_keys)
    x, info = krylov.fgmres(A, f, restart=n, rtol=1e-12)
    assert info["iters"] <= n
    assert np.abs(x - np.linalg.solve(A.toarray(), f)).max() < 1e-8 * np.abs(x).max()


def test_ilu0_identity_on_pattern():
    bd, E, Om, A, P = C.matrices("sphere", (1.0,), 3, 0.2, 3, 1.0)
    idx = np.arange(min(400, bd.n_active))
    Aj = sp.csr_matrix(A[idx][:, idx])
    L, U = schwarz.ilu0(Aj)
    LU = ((L + sp.identity(idx.size)) @ U).tocsr()
    Ad = Aj.toarray()
    mask = Aj.toarray() != 0
    mask |= sp.csr_matrix((np.ones(Aj.nnz), Aj.indices, Aj.indptr), shape=Aj.shape).toarray() != 0
    assert np.abs((LU.toarray() - Ad)[mask]).max() < 1e-9 * np.abs(Ad).max()
    # L and U live on the pattern
    assert set(zip(*sp.triu(U).nonzero())) <= set(zip(*np.nonzero(mask)))


def test_ilu0_without_fill_is_exact_lu():
    n = 50
    rng = np.random.default_rng(2)
    T = sp.diags([rng.uniform(-1, 0, n - 1), rng.uniform(4, 5, n), rng.uniform(-1, 0, n - 1)],
                 [-1, 0, 1], format="csr")
    L, U = schwarz.ilu0(T)
    Pm, Ld, Ud = sla.lu(T.toarray())
    assert np.allclose(Pm, np.eye(n))
    assert np.abs((L + sp.identity(n)).toarray() - Ld).max() < 1e-14
    assert np.abs(U.toarray() - Ud).max() < 1e-13


def _sphere_ras(kind="ras", n_parts=8, h=0.1, alpha=4.0, alpha_cross=20.0, subsolver="ilu0", c=1.0):
    bd, E, Om, A, P = C.matrices("sphere", (1.0,), 3, h, 3, c)
    S = schwarz.build_schwarz(A, P, bd.cp_active, bd.active_keys, h, n_parts, 2.0, kind=kind,
                              alpha=alpha, alpha_cross=alpha_cross, subsolver=subsolver)
    return bd, A, S


def test_ras_partition_of_unity_and_ownership():
    bd, A, S = _sphere_ras()
    n = bd.n_active
    cover = np.zeros(n, dtype=int)
    for j, idx in enumerate(S.omegas):
        own = S.owner[idx] == j
        cover[idx[own]] += 1
        assert (S.owner == j).sum() == own.sum()   # every owned node lies in its Omega_j
    assert (cover == 1).all()
    # restricted recombination of R_j x gives x back
    x = np.random.default_rng(0).standard_normal(n)
    z = np.zeros(n)
    for j, idx in enumerate(S.omegas):
        own = S.owner[idx] == j
        z[idx[own]] = x[idx][own]
    assert np.array_equal(z, x)
    sizes = np.bincount(S.owner)
    assert sizes.min() > 0.7 * sizes.mean()


def test_single_subdomain_exact_lu_is_inverse():
    bd, A, S = _sphere_ras(n_parts=1, subsolver="lu")
    f = inputs.sphere_y4(bd.cp_active, 2) * 21.0
    x, info = krylov.fgmres(A, f, M=S.apply, rtol=1e-10)
    assert info["iters"] == 1 and info["converged"]


def test_oras_large_alpha_is_ras():
    bd, A, S1 = _sphere_ras(kind="ras")
    _, _, S2 = _sphere_ras(kind="oras", alpha=1e300, alpha_cross=1e300)
    r = np.random.default_rng(1).standard_normal(bd.n_active)
    z1, z2 = S1.apply(r), S2.apply(r)
    assert np.abs(z1 - z2).max() <= 1e-13 * np.abs(z1).max()
    _, _, S3 = _sphere_ras(kind="oras")
    assert np.abs(S3.apply(r) - z1).max() > 1e-6 * np.abs(z1).max()


def test_preconditioners_leave_solution_unchanged_and_help():
    """Every preconditioner converges to the same solution; RAS with ILU(0) and ORAS with
    exact local solves cut the iteration count. (ORAS with ILU(0) local solves can be worse
    than no preconditioner: the paper reports this ILU/Robin interaction, Sec. 4.1.1.)"""
    bd, A, Sr = _sphere_ras(kind="ras")
    _, _, So = _sphere_ras(kind="oras")
    _, _, Srl = _sphere_ras(kind="ras", subsolver="lu")
    _, _, Sol = _sphere_ras(kind="oras", subsolver="lu")
    f = inputs.sphere_y4(bd.cp_active, 2) * 21.0
    x0, i0 = krylov.fgmres(A, f, rtol=1e-11)
    s = np.abs(x0).max()
    its = {}
    for name, S in (("ras", Sr), ("oras", So), ("ras_lu", Srl), ("oras_lu", Sol)):
        x, info = krylov.fgmres(A, f, M=S.apply, rtol=1e-11, max_it=2000)
        assert info["converged"] and np.abs(x - x0).max() < 1e-9 * s, name
        its[name] = info["iters"]
    assert its["ras"] < i0["iters"] and its["ras_lu"] < its["ras"]
    assert its["oras_lu"] <= its["ras_lu"]


def test_adjoint_gradients_exact_central_differences():
    bd, E, Om, A, P = C.matrices("circle", (1.0,), 2, 0.1, 3, 1.5)
    n = bd.n_active
    f = inputs.normal(1, 0, bd.active_keys)
    ut = inputs.normal(1, 1, bd.active_keys)
    L, u, gf, gc = adjoint.quadratic_loss_grads(A, f, ut)
    Ld, ud, gfd, gcd = adjoint.quadratic_loss_grads(A, f, ut, dense=True)
    assert abs(L - Ld) < 1e-10 * L and np.abs(gf - gfd).max() < 1e-10 * np.abs(gf).max()
    eps = max(1.0, np.abs(f).max())
    for i in np.random.default_rng(0).choice(n, 8, replace=False):
        e = np.zeros(n)
        e[i] = eps
        fd = (adjoint.quadratic_loss_grads(A, f + e, ut)[0]
              - adjoint.quadratic_loss_grads(A, f - e, ut)[0]) / (2 * eps)
        assert abs(fd - gf[i]) <= 1e-8 * max(abs(gf[i]), 1e-3 * np.abs(gf).max())
    # derivative in c: A(c) = A + (c' - c) I
    ec = 1e-4 * 1.5
    Ip = sp.identity(n, format="csr")
    fd = (adjoint.quadratic_loss_grads(A + ec * Ip, f, ut)[0]
          - adjoint.quadratic_loss_grads(A - ec * Ip, f, ut)[0]) / (2 * ec)
    assert abs(fd - gc) <= 1e-6 * abs(gc)
    # transpose identity on the assembled operator
    x, y = inputs.normal(2, 0, bd.active_keys), inputs.normal(2, 1, bd.active_keys)
    assert abs(np.dot(A @ x, y) - np.dot(x, adjoint.transpose_apply(A, y))) < 1e-12 * np.abs(A @ x).sum()


def test_gray_scott_uniform_state_follows_reaction_ode():
    bd, E, Om, A0, P = C.matrices("circle", (1.0,), 2, 0.1, 3, 0.0)
    mu, dt, F, k = (2e-5, 1e-5), 1.0, 0.04, 0.06
    n = bd.n_active
    Ip = sp.identity(n, format="csr")
    Au = (A0 + (1.0 / (mu[0] * dt)) * Ip).tocsc()
    Av = (A0 + (1.0 / (mu[1] * dt)) * Ip).tocsc()
    import scipy.sparse.linalg as spla
    su, sv = spla.factorized(Au), spla.factorized(Av)
    u, v = np.full(n, 0.7), np.full(n, 0.2)
    uu, vv = 0.7, 0.2
    for _ in range(5):
        u, v = reaction.imex_step(su, sv, u, v, F, k, mu, dt)
        Ru, Rv = reaction.gray_scott_reaction(uu, vv, F, k)
        uu, vv = uu + dt * Ru, vv + dt * Rv
    assert np.abs(u - uu).max() < 1e-10 and np.abs(v - vv).max() < 1e-10
    # (1, 0) is a fixed point
    u1, v1 = reaction.imex_step(su, sv, np.ones(n), np.zeros(n), F, k, mu, dt)
    assert np.abs(u1 - 1).max() < 1e-10 and np.abs(v1).max() < 1e-12


def test_rcm_textbook_cases():
    """Reverse Cuthill-McKee: a path graph given in shuffled order comes back as a path
    (bandwidth 1), starting from a least-degree end; a shuffled banded matrix regains a
    narrow band; the result is always a permutation."""
    rng = np.random.default_rng(3)
    n = 40
    P = sp.diags([np.ones(n - 1), np.ones(n), np.ones(n - 1)], [-1, 0, 1], format="csr")
    q = rng.permutation(n)
    Pq = sp.csr_matrix(P[q][:, q])
    perm = schwarz.rcm_order(Pq)
    assert np.array_equal(np.sort(perm), np.arange(n))
    B = sp.csr_matrix(Pq[perm][:, perm])
    rows, cols = B.nonzero()
    assert np.abs(rows - cols).max() == 1
    # banded (bandwidth 5) random pattern, shuffled
    n = 200
    M = sp.random(n, n, density=1.0, random_state=1, format="csr")
    M = sp.csr_matrix(sp.triu(sp.tril(M, 5), -5) + sp.identity(n))
    q = rng.permutation(n)
    Mq = sp.csr_matrix(M[q][:, q])
    r0, c0 = Mq.nonzero()
    perm = schwarz.rcm_order(Mq)
    r1, c1 = sp.csr_matrix(Mq[perm][:, perm]).nonzero()
    assert np.abs(r1 - c1).max() <= 12 < np.abs(r0 - c0).max()
    # the empty graph: least (degree, index) order reversed
    assert np.array_equal(schwarz.rcm_order(sp.identity(5, format="csr")), np.arange(5)[::-1])


def test_distance_order_cases_and_short_chains():
    """Distance order: decreasing distance, equal distances keep their index order; on
    a real subdomain the ILU(0) forward sweep's longest dependency chain is short (rows
    couple only to rows at larger or equal distance before them) while RCM's is long."""
    assert np.array_equal(schwarz.distance_order(np.array([0.3, 0.1, 0.3, 0.2])), [0, 2, 3, 1])
    assert np.array_equal(schwarz.distance_order(np.zeros(4)), np.arange(4))
    bd, E, O, A, P = C.matrices("sphere", (1.0,), 3, 0.1, 3, 1.0)
    dist = surfaces.distance(OB.coords(bd.active_ijk, bd.lo, bd.h), bd.cp_active)
    owner, blo, bhi = schwarz.rcb_partition(bd.cp_active, 2)
    idx = schwarz.overlap_sets(bd.cp_active, blo, bhi, 0.2, bd.active_keys)[0]
    Aj = sp.csr_matrix(sp.csr_matrix(A)[idx][:, idx])

    def chain(perm):
        L = sp.csr_matrix(sp.tril(sp.csr_matrix(Aj[perm][:, perm]), k=-1))
        lev = np.zeros(L.shape[0], dtype=np.int64)
        for i in range(L.shape[0]):
            js = L.indices[L.indptr[i]:L.indptr[i + 1]]
            lev[i] = lev[js].max() + 1 if js.size else 0
        return lev.max() + 1

    pd = schwarz.distance_order(dist[idx])
    assert np.all(np.diff(dist[idx][pd]) <= 0)
    assert 3 * chain(pd) < chain(schwarz.rcm_order(Aj))


def _toy_9pt_grid():
    """4 x 4 grid of points (x, y), keys 4x + y, a 9-point stencil matrix with
    diagonal 10, edge couplings -1 and corner couplings -0.5."""
    pts = np.array([(x, y) for x in range(4) for y in range(4)], dtype=np.float64)
    n = len(pts)
    A = np.zeros((n, n))
    for i, (x, y) in enumerate(pts):
        A[i, i] = 10.0
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                if (dx, dy) == (0, 0) or not (0 <= x + dx < 4 and 0 <= y + dy < 4):
                    continue
                k = int((x + dx) * 4 + (y + dy))
                A[i, k] = -1.0 if dx == 0 or dy == 0 else -0.5
    return pts, sp.csr_matrix(A)


def test_oras_robin_alpha_selection_hand_worked():
    """ORAS Robin lumping on a case worked out by hand (reading of eq. transRob).

    RCB of the 4 x 4 points into 4 parts cuts x at 2, then y at 2: owners are the
    quadrants {x<2,y<2}, {x<2,y>=2}, {x>=2,y<2}, {x>=2,y>=2}. With overlap 0 the
    closed boxes give Omega_0 = {x<=2, y<=2} and Omega_3 = {x>=2, y>=2}. Dropped
    couplings and their owners, h = 0.5 (1/(1 + 4h) = 1/3, 1/(1 + 20h) = 1/11):
      Omega_0 row (0,2): (0,3) edge, (1,3) corner -> owner {1}        -> 10 - 1.5/3
      Omega_0 row (1,2): (0,3), (2,3) corners, (1,3) edge -> {1, 3}   -> 10 - 2/11
      Omega_0 row (2,2): (1,3),(3,3),(3,1) corners, (2,3),(3,2) edges
                         -> owners {1, 2, 3}                          -> 10 - 3.5/11
      Omega_0 row (2,0): (3,0) edge, (3,1) corner -> {2}              -> 10 - 1.5/3
      Omega_0 row (2,1): (3,0),(3,2) corners, (3,1) edge -> {2, 3}    -> 10 - 2/11
      Omega_3 row (2,2): (1,1),(1,3),(3,1) corners, (1,2),(2,1) edges
                         -> {0, 1, 2}                                 -> 10 - 3.5/11
      Omega_3 rows (2,3), (3,2): one edge + one corner, one owner     -> 10 - 1.5/3
    Swapping alpha and alpha_cross, counting one owner as a cross point, or
    dropping h from 1 + alpha h each change at least one of these values.
    """
    pts, A = _toy_9pt_grid()
    keys = (pts[:, 0] * 4 + pts[:, 1]).astype(np.int64)
    S = schwarz.build_schwarz(A, A, pts, keys, 0.5, 4, 0.0, kind="oras", alpha=4.0, alpha_cross=20.0,
                              subsolver="lu")
    quad = (pts[:, 0] >= 2).astype(int) * 2 + (pts[:, 1] >= 2).astype(int)
    assert np.array_equal(S.owner, quad)
    want0 = {(0, 0): 10.0, (0, 1): 10.0, (0, 2): 10.0 - 1.5 / 3, (1, 0): 10.0, (1, 1): 10.0,
             (1, 2): 10.0 - 2.0 / 11, (2, 0): 10.0 - 1.5 / 3, (2, 1): 10.0 - 2.0 / 11, (2, 2): 10.0 - 3.5 / 11}
    want3 = {(2, 2): 10.0 - 3.5 / 11, (2, 3): 10.0 - 1.5 / 3, (3, 2): 10.0 - 1.5 / 3, (3, 3): 10.0}
    for j, want in ((0, want0), (3, want3)):
        idx = S.omegas[j]
        got = {tuple(int(v) for v in pts[i]): S.local[j].diagonal()[li] for li, i in enumerate(idx)}
        assert set(got) == set(want)
        for q, v in want.items():
            assert abs(got[q] - v) <= 1e-15 * 10, (j, q, got[q], v)
        # off-diagonal entries of the local matrix are A's own
        Ad = A.toarray()[np.ix_(idx, idx)]
        Ld = S.local[j].toarray()
        off = ~np.eye(idx.size, dtype=bool)
        assert np.array_equal(Ld[off], Ad[off])


def test_oras_local_rows_follow_robin_substitution_sphere():
    """On a CPM band (sphere h = 0.2, p = 3, 8 parts, overlap 2h) every local ORAS row
    equals A's row applied to the local vector extended outside Omega_j by the
    discrete Robin relation u_k = u_i / (1 + alpha_i h), alpha_i chosen by the
    number of distinct owners of the row's dropped columns (found here from the
    dense matrix by set operations)."""
    bd, E, Om, A, P = C.matrices("sphere", (1.0,), 3, 0.2, 3, 1.0)
    h, al, alx = 0.2, 4.0, 20.0
    S = schwarz.build_schwarz(A, P, bd.cp_active, bd.active_keys, h, 8, 2.0, kind="oras", alpha=al,
                              alpha_cross=alx, subsolver="lu")
    Ad = A.toarray()
    Pd = P.toarray() != 0
    rng = np.random.default_rng(11)
    n_cross = n_single = 0
    for j, idx in enumerate(S.omegas):
        inside = set(int(i) for i in idx)
        uloc = rng.standard_normal(idx.size)
        got = S.local[j] @ uloc
        for li, i in enumerate(idx):
            dropped = [k for k in np.nonzero(Pd[i])[0] if int(k) not in inside]
            owners = {int(S.owner[k]) for k in dropped}
            assert j not in owners
            a = alx if len(owners) >= 2 else al
            w = np.zeros(A.shape[0])
            w[idx] = uloc
            for k in dropped:
                w[k] = uloc[li] / (1.0 + a * h)
            want = Ad[i] @ w
            assert abs(got[li] - want) <= 1e-12 * (np.abs(Ad[i]) @ np.abs(w) + 1e-300)
            n_cross += len(owners) >= 2
            n_single += len(owners) == 1
    assert n_cross > 0 and n_single > 0


def test_two_level_coarse_matrix_brute_force_and_galerkin():
    """A0[j, k] = sum of A over (rows owned by j) x (columns owned by k), by explicit loops on a
    small band; the hybrid correction leaves a residual with zero coarse component
    (R0 (r - A z_c) = 0); P = R0^T A0^-1 R0 A is a projection that fixes the coarse space."""
    bd, E, Om, A, P = C.matrices("circle", (1.0,), 2, 0.1, 2, 1.0)
    one = schwarz.build_schwarz(A, P, bd.cp_active, bd.active_keys, 0.1, 4, 2.0, kind="ras", subsolver="lu")
    tl = schwarz.build_two_level(A, one, "hybrid")
    Ad = A.toarray()
    owner = one.owner
    for j in range(4):
        for k in range(4):
            s = 0.0
            for i in np.nonzero(owner == j)[0]:
                for l_ in np.nonzero(owner == k)[0]:
                    s += Ad[i, l_]
            assert abs(tl.A0[j, k] - s) <= 1e-12 * np.abs(Ad).sum()
    r = np.random.default_rng(5).standard_normal(bd.n_active)
    zc = tl.coarse(r)
    assert np.abs(tl.R0 @ (r - A @ zc)).max() <= 1e-12 * np.abs(tl.R0 @ r).max()
    Pm = lambda x: tl.coarse(A @ x)
    x = np.random.default_rng(6).standard_normal(bd.n_active)
    assert np.abs(Pm(Pm(x)) - Pm(x)).max() <= 1e-12 * np.abs(Pm(x)).max()
    e = np.random.default_rng(7).standard_normal(4)
    assert np.abs(Pm(tl.R0.T @ e) - tl.R0.T @ e).max() <= 1e-12 * np.abs(e).max()


def test_two_level_keeps_iterations_flat_under_weak_scaling():
    """Unit sphere, exact local solves, subdomains growing with the unknowns (h = 0.1 with 8
    boxes, h = 0.05 with 32): one-level RAS needs more FGMRES iterations as N_S grows, the
    hybrid two-level preconditioner fewer, with a smaller growth; the solution is unchanged."""
    res = {}
    for h, ns in ((0.1, 8), (0.05, 32)):
        bd, E, Om, A, P = C.matrices("sphere", (1.0,), 3, h, 3, 1.0)
        f = 21.0 * inputs.sphere_y4(bd.cp_active, 2)
        one = schwarz.build_schwarz(A, P, bd.cp_active, bd.active_keys, h, ns, 2.0, kind="ras", subsolver="lu")
        tl = schwarz.build_two_level(A, one, "hybrid")
        x1, i1 = krylov.fgmres(A, f, M=one.apply, rtol=1e-8, max_it=3000)
        x2, i2 = krylov.fgmres(A, f, M=tl.apply, rtol=1e-8, max_it=3000)
        assert i1["converged"] and i2["converged"]
        assert np.abs(x1 - x2).max() <= 1e-6 * np.abs(x1).max()
        res[h] = (i1["iters"], i2["iters"])
    print(res)
    (a1, a2), (b1, b2) = res[0.1], res[0.05]
    assert a2 <= a1 and b2 < b1
    assert b2 - a2 < b1 - a1
