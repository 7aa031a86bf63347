"""Pins of the oracle's two-level column semicoarsening preconditioner (no GPU).

Each step is pinned by something other than its own formula: the column block LU against a
dense solve, the vertical weights by multiplying back, the aggregation by a worked example
and by the properties its rules imply, the Chebyshev recurrence by its closed-form error
polynomial on the eigenvectors, the V-cycle by its error-propagation operator, and the whole
preconditioner by the cases where it must be exact.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from fo_inputs import config0_slab, ellipse_mesh, ExtrudedMesh, smooth_velocity
from fo_inputs.meshgen import _dome_fields
from oracle import fo_oracle as fo
from oracle import mdsc


def _cap(n_points, seed=3, n_layers=6):
    rng = np.random.default_rng(seed)
    a, b = 60e3, 35e3
    xy, tri = ellipse_mesh(n_points, a, b, rng)
    s, H, beta = _dome_fields(xy, a, b, rng, 2000.0, 300.0, 500.0, 1.0, 8e3, 30e3)
    m = ExtrudedMesh("wedge", xy, tri, s, H, beta, np.linspace(0, 1, n_layers + 1), A=1e-16)
    return m, smooth_velocity(m, rng)


@pytest.fixture(scope="module")
def cap():
    m, U = _cap(400)
    _, J = fo.assemble(m, U)
    return m, J.tocsr()


@pytest.fixture(scope="module")
def slab():
    m, U = config0_slab()
    _, J = fo.assemble(m, U)
    return m, J.tocsr()


def _block_tridiag(rng, V, L1):
    """Random symmetric positive definite block-tridiagonal columns [V, 2 L1, 2 L1]."""
    nb = 2 * L1
    B = np.zeros((V, nb, nb))
    for v in range(V):
        M = rng.normal(size=(nb, nb))
        band = np.abs(np.subtract.outer(np.arange(nb) // 2, np.arange(nb) // 2)) <= 1
        S = (M @ M.T) * band
        B[v] = S + nb * np.eye(nb)
    return B


def test_column_factors_solve_the_columns():
    rng = np.random.default_rng(0)
    B = _block_tridiag(rng, 7, 6)
    r = rng.normal(size=7 * 12)
    want = np.concatenate([np.linalg.solve(B[v], r[12 * v:12 * v + 12]) for v in range(7)])
    z64 = mdsc.column_solve(mdsc.column_factors(B, store=np.float64), r)
    assert np.abs(z64 - want).max() <= 1e-12 * np.abs(want).max()
    z32 = mdsc.column_solve(mdsc.column_factors(B), r)       # FP32-stored factors
    cond = max(np.linalg.cond(B[v]) for v in range(7))
    assert np.abs(z32 - want).max() <= 4 * cond * 6e-8 * np.abs(want).max()
    assert np.abs(z32 - want).max() > 0          # the rounding is really applied


def test_vertical_weights_multiply_back(cap):
    m, J = cap
    blocks = mdsc.column_blocks(m, J)
    W = mdsc.vertical_weights(blocks)
    V, L1 = W.shape[:2]
    for c in range(2):
        w = W[:, :, :, c].reshape(V, 2 * L1)
        Bw = np.einsum("vij,vj->vi", blocks, w)
        # B_v w = alpha_v e_c: constant alpha > 0 on component c, zero on the other
        comp = Bw.reshape(V, L1, 2)
        alpha = comp[:, 0, c]
        assert np.all(alpha > 0)
        scale = np.abs(blocks).max(axis=(1, 2)) * np.abs(w).max(axis=1)
        assert np.all(np.abs(comp[:, :, c] - alpha[:, None]).max(axis=1) <= 1e-10 * scale)
        assert np.all(np.abs(comp[:, :, 1 - c]).max(axis=1) <= 1e-10 * scale)
        assert np.allclose(W[:, :, c, c].mean(axis=1), 1.0, rtol=0, atol=1e-13)


def test_vertical_weights_fallback_on_indefinite_column():
    rng = np.random.default_rng(1)
    B = _block_tridiag(rng, 3, 4)
    B[1] = -B[1]                          # negative definite: B^-1 e_c has negative mean
    W = mdsc.vertical_weights(B)
    e = np.zeros((4, 2, 2))
    e[:, 0, 0] = e[:, 1, 1] = 1.0
    assert np.array_equal(W[1], e)
    assert not np.array_equal(W[0], e)


def test_plane_graph_is_the_column_coupling_of_the_jacobian(cap):
    m, J = cap
    nb = 2 * (m.n_layers + 1)
    C = sp.coo_matrix(J)
    pairs = set(zip((C.row // nb).tolist(), (C.col // nb).tolist()))
    nbrs = mdsc.plane_graph(m)
    assert pairs == {(v, w) for v in range(m.n_verts) for w in nbrs[v]}


def test_aggregation_worked_example():
    # path 0-1-2-3-4-5-6, then two isolated vertices 7, 8, then a triangle 9-10-11
    path = [[0, 1], [0, 1, 2], [1, 2, 3], [2, 3, 4], [3, 4, 5], [4, 5, 6], [5, 6]]
    nbrs = path + [[7], [8], [9, 10, 11], [9, 10, 11], [9, 10, 11]]
    agg, n_agg = mdsc.aggregate(nbrs)
    # pass 1: root 0 takes {0,1}; 2 has assigned neighbour 1; root 3 takes {2,3,4};
    # 5 has 4; root 6 takes {5,6}; 7, 8 open an isolated group; root 9 takes {9,10,11}
    assert agg.tolist() == [0, 0, 1, 1, 1, 2, 2, 3, 3, 4, 4, 4] and n_agg == 5
    # a vertex skipped in pass 1 can still become part of a later root's aggregate: 2 is
    # next to 0's aggregate, but root 3 (neighbours 2, 4, 5 all free) takes it
    nbrs = [[0, 1], [0, 1, 2], [1, 2, 3], [2, 3, 4, 5], [3, 4], [3, 5]]
    agg, n_agg = mdsc.aggregate(nbrs)
    assert agg.tolist() == [0, 0, 1, 1, 1, 1] and n_agg == 2
    # pass 2: roots 0 {0, 1} and 3 {2, 3, 4}; 5 (neighbour 4 assigned) is left to pass 2 and
    # joins the aggregate of 4, its lowest-numbered neighbour assigned in pass 1
    nbrs = [[0, 1], [0, 1, 2], [1, 2, 3], [2, 3, 4], [3, 4, 5], [4, 5]]
    agg, _ = mdsc.aggregate(nbrs)
    assert agg.tolist() == [0, 0, 1, 1, 1, 1]
    # pass 2 takes the lowest-numbered assigned neighbour: edges 0-1, 2-3, 1-4, 3-4; roots 0
    # {0, 1} and 2 {2, 3}; 4 (neighbours 1 and 3, both assigned) joins 1's aggregate
    nbrs = [[0, 1], [0, 1, 4], [2, 3], [2, 3, 4], [1, 3, 4]]
    agg, _ = mdsc.aggregate(nbrs)
    assert agg.tolist() == [0, 0, 1, 1, 0]


def test_isolated_vertices_grouped_by_eight():
    agg, n_agg = mdsc.aggregate([[v] for v in range(19)])
    assert agg.tolist() == [0] * 8 + [1] * 8 + [2] * 3 and n_agg == 3


def test_aggregation_properties_on_a_mesh_graph(cap):
    m, _ = cap
    nbrs = mdsc.plane_graph(m)
    agg, n_agg = mdsc.aggregate(nbrs)
    assert agg.min() == 0 and agg.max() == n_agg - 1 and len(np.unique(agg)) == n_agg
    adj = [set(l) for l in nbrs]
    members = [np.flatnonzero(agg == a) for a in range(n_agg)]
    roots = []
    for a, mem in enumerate(members):
        # connected: a breadth-first search inside the aggregate reaches every member
        seen, todo = {mem[0]}, [mem[0]]
        while todo:
            x = todo.pop()
            for y in adj[x]:
                if agg[y] == a and y not in seen:
                    seen.add(y)
                    todo.append(y)
        assert seen == set(mem.tolist())
        # its root (lowest member whose whole neighbourhood is inside) exists
        r = [v for v in mem if adj[v] <= set(mem.tolist())]
        assert r
        roots.append(min(r))
    # roots are at graph distance >= 3 from each other
    for r in roots:
        two = set().union(*[adj[x] for x in adj[r]])
        assert not (set(roots) - {r}) & two
    assert n_agg < len(nbrs) / 3


def test_galerkin_blocks_are_sums_over_aggregate_pairs(cap):
    m, J = cap
    H = mdsc.Hierarchy(m, J)
    lv = H.levels[0]
    A, agg, n_agg = lv["A"].toarray(), lv["agg"], lv["n_agg"]
    want = np.zeros((2 * n_agg, 2 * n_agg))
    for v in range(len(agg)):
        for w in range(len(agg)):
            want[2 * agg[v]:2 * agg[v] + 2, 2 * agg[w]:2 * agg[w] + 2] += A[2 * v:2 * v + 2, 2 * w:2 * w + 2]
    got = (lv["T"].T @ lv["A"] @ lv["T"]).toarray()
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
    # the plane operator of the collapse is P0^T J P0 entry by entry
    P0 = H.P0.toarray()
    A1 = P0.T @ J.toarray() @ P0
    assert np.abs(A1 - A).max() <= 1e-12 * np.abs(A1).max()


def test_gershgorin_bound():
    rng = np.random.default_rng(2)
    # nonnegative D^-1 A with constant row sums: the bound is the Perron root
    n = 12
    M = rng.uniform(0.1, 1.0, size=(2 * n, 2 * n))
    M /= M.sum(axis=1, keepdims=True)
    A = sp.csr_matrix(M * 3.5)
    Dinv = mdsc.diag_block_inverse(A)
    DA = (Dinv @ A).toarray()
    g = mdsc.gershgorin(A, Dinv)
    assert abs(g - np.abs(DA).sum(axis=1).max()) <= 1e-14 * g
    S = rng.normal(size=(2 * n, 2 * n))
    A = sp.csr_matrix(S @ S.T + 2 * n * np.eye(2 * n))
    Dinv = mdsc.diag_block_inverse(A)
    rho = np.abs(np.linalg.eigvals((Dinv @ A).toarray())).max()
    assert mdsc.gershgorin(A, Dinv) >= rho * (1 - 1e-12)


def test_chebyshev_matches_its_error_polynomial():
    """After k steps from x0 the error is p_k(D^-1 A) e0 with
    p_k(t) = T_k((theta - t) / delta) / T_k(theta / delta)."""
    rng = np.random.default_rng(4)
    n = 10
    S = rng.normal(size=(2 * n, 2 * n))
    A = S @ S.T + 0.5 * np.eye(2 * n)
    Asp = sp.csr_matrix(A)
    Dinv = mdsc.diag_block_inverse(Asp)
    g = mdsc.gershgorin(Asp, Dinv)
    b = rng.normal(size=2 * n)
    x0 = rng.normal(size=2 * n)
    xs = np.linalg.solve(A, b)
    lam, X = np.linalg.eig((Dinv @ Asp).toarray())
    lam, X = lam.real, X.real
    for deg in (1, 2, 3):
        for ratio in (30.0, 4.0):
            lo = g / ratio
            theta, delta = 0.5 * (g + lo), 0.5 * (g - lo)
            Tk = np.polynomial.chebyshev.Chebyshev.basis(deg)
            p = Tk((theta - lam) / delta) / Tk(theta / delta)
            e = X @ (p * np.linalg.solve(X, x0 - xs))
            got = mdsc.chebyshev(Asp, Dinv, g, b, x0, degree=deg, ratio=ratio)
            assert np.abs(got - (xs + e)).max() <= 1e-10 * np.abs(xs).max(), (deg, ratio)


def _cheb_error_operator(A, Dinv, g, degree):
    """p(D^-1 A) with p(t) = T_k((theta - t)/delta) / T_k(theta/delta) on [g/30, g]."""
    n = A.shape[0]
    lo = g / mdsc.CHEB_RATIO
    theta, delta = 0.5 * (g + lo), 0.5 * (g - lo)
    Y = (theta * np.eye(n) - Dinv @ A) / delta
    Tk = np.polynomial.chebyshev.Chebyshev.basis(degree).convert(kind=np.polynomial.Polynomial).coef
    P = sum(c * np.linalg.matrix_power(Y, i) for i, c in enumerate(Tk))
    return P / np.polynomial.chebyshev.Chebyshev.basis(degree)(theta / delta)


def test_vcycle_error_propagation(slab):
    """One smoothing level and an exact coarsest level: the V-cycle B satisfies
    I - B A = S (I - T A_c^-1 T^T A) S with S = p_2(D^-1 A) the smoother's error operator."""
    m, J = slab
    H = mdsc.Hierarchy(m, J)
    assert len(H.levels) == 1
    lv = H.levels[0]
    A, Dinv, g, T = lv["A"].toarray(), lv["Dinv"].toarray(), lv["g"], lv["T"].toarray()
    n = A.shape[0]
    lo = g / mdsc.CHEB_RATIO
    theta, delta = 0.5 * (g + lo), 0.5 * (g - lo)
    DA = Dinv @ A
    # p_2(t) = T_2((theta - t)/delta) / T_2(theta/delta), T_2(s) = 2 s^2 - 1
    Y = (theta * np.eye(n) - DA) / delta
    S = (2 * Y @ Y - np.eye(n)) / (2 * (theta / delta) ** 2 - 1)
    Ac = T.T @ A @ T
    E = S @ (np.eye(n) - T @ np.linalg.solve(Ac, T.T @ A)) @ S
    B = np.column_stack([H.vcycle(col) for col in np.eye(n)])
    assert np.abs((np.eye(n) - B @ A) - E).max() <= 1e-9


def test_vcycle_error_propagation_two_levels():
    """Two smoothing levels (degree 2, then degree 1) above the exact coarsest level: the
    recursion I - B_0 A_0 = S_0 (I - T_0 B_1 T_0^T A_0) S_0 with
    I - B_1 A_1 = S_1 (I - T_1 A_c^-1 T_1^T A_1) S_1."""
    m, U = _cap(600, seed=3, n_layers=1)
    _, J = fo.assemble(m, U)
    H = mdsc.Hierarchy(m, J.tocsr())
    assert len(H.levels) == 2
    l0, l1 = H.levels
    A0, A1 = l0["A"].toarray(), l1["A"].toarray()
    T0, T1 = l0["T"].toarray(), l1["T"].toarray()
    S0 = _cheb_error_operator(A0, l0["Dinv"].toarray(), l0["g"], 2)
    S1 = _cheb_error_operator(A1, l1["Dinv"].toarray(), l1["g"], 1)
    Ac = T1.T @ A1 @ T1
    n1 = A1.shape[0]
    B1 = np.linalg.solve(A1.T, (np.eye(n1) - S1 @ (np.eye(n1) - T1 @ np.linalg.solve(Ac, T1.T @ A1)) @ S1).T).T
    n0 = A0.shape[0]
    E0 = S0 @ (np.eye(n0) - T0 @ B1 @ T0.T @ A0) @ S0
    B = np.column_stack([H.vcycle(col) for col in np.eye(n0)])
    assert np.abs((np.eye(n0) - B @ A0) - E0).max() <= 1e-8


def test_apply_is_exact_on_the_coarse_range_and_for_column_operators(cap):
    m, J = cap
    rng = np.random.default_rng(5)
    # plane small enough to be solved exactly: the residual left by the coarse correction is
    # orthogonal to the coarse space, and an error in the range of P0 is removed exactly
    small, Us = _cap(60, seed=6, n_layers=4)
    _, Js = fo.assemble(small, Us)
    H = mdsc.Hierarchy(small, Js, store=np.float64)
    assert not H.levels
    r = rng.normal(size=small.n_dofs)
    y = np.linalg.solve(H.A_coarse, H.P0.T @ r)
    assert np.abs(H.P0.T @ (r - H.JP @ y)).max() <= 1e-10 * np.abs(H.P0.T @ r).max()
    y0 = rng.normal(size=2 * small.n_verts)
    x0 = H.P0 @ y0
    assert np.abs(H.apply(Js @ x0) - x0).max() <= 1e-9 * np.abs(x0).max()
    # a Jacobian without coupling between columns: the preconditioner is its inverse (up to
    # the FP32 factors), through every level of the hierarchy
    nb = 2 * (m.n_layers + 1)
    C = sp.coo_matrix(J)
    keep = (C.row // nb) == (C.col // nb)
    Jc = sp.csr_matrix((C.data[keep], (C.row[keep], C.col[keep])), shape=J.shape)
    Hc = mdsc.Hierarchy(m, Jc, store=np.float64)
    assert Hc.levels
    r = rng.normal(size=m.n_dofs)
    want = sp.linalg.spsolve(Jc.tocsc(), r)
    assert np.abs(Hc.apply(r) - want).max() <= 1e-9 * np.abs(want).max()
    # with the parts stored in FP32 it stays the inverse to the FP32 rounding
    Hc32 = mdsc.Hierarchy(m, Jc)
    assert np.abs(Hc32.apply(r) - want).max() <= 1e-5 * np.abs(want).max()


def test_two_level_cuts_gmres_iterations(cap):
    """What the hierarchy is for: fewer GMRES iterations than the column smoother alone."""
    import scipy.sparse.linalg as spla
    m, J = cap
    H = mdsc.Hierarchy(m, J)
    b = np.random.default_rng(7).normal(size=m.n_dofs)
    B = mdsc.column_factors(mdsc.column_blocks(m, J))
    counts = []
    for prec in (lambda r: mdsc.column_solve(B, r), H.apply):
        its = [0]
        M = spla.LinearOperator(J.shape, matvec=prec)
        _, info = spla.gmres(J, b, M=M, rtol=1e-8, restart=200, maxiter=2,
                             callback=lambda _: its.__setitem__(0, its[0] + 1), callback_type="pr_norm")
        assert info == 0
        counts.append(its[0])
    assert counts[1] < 0.8 * counts[0], counts
