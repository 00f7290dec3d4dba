"""FP64 oracle of the blockBP update: imaginary time evolution of a PEPS
with block-BP environments (App. B of Guo, Poletti, Arad; Sec. II, "blockBP
update").

TEST INFRASTRUCTURE, like the rest of ``oracle/``: plain NumPy, only the
tests use it, and it shares no code with the GPU library.

One step applies the first-order Trotter gates ``G = exp(-h dtau)`` of every
nearest-neighbour bond (Eq. (Ut)), horizontal bonds row by row, then vertical
bonds column by column.  The block-BP messages are converged before the step
and stay fixed through it; each gate sees the current tensors of its region
(the bond's block, or the union of the two blocks it joins) with those
messages as the boundary, contracted by boundary MPSs as for observables.
A gate is applied by minimising ``|| psi' - G psi ||^2`` over the two
tensors of its bond (App. B), in the reduced form of the full update: the
two tensors are split by QR (the one on the left or top) and LQ (the other)
into an isometry on their outer legs and a small reduced tensor holding the
physical index and the shared bond; the environment of the two reduced
tensors is the two-site reduced density matrix of the network in which the
two sites carry their isometries' bond as the physical index; the reduced
tensors are then fitted by alternating least squares.

Readings (the paper leaves these open):
* gate order: horizontal bonds by rows (y, then x ascending), then vertical
  bonds by columns (x, then y ascending);
* the reduced tensors: the first site's legs other than the shared one, at
  their true dimensions (1 on the lattice edge, D inside), form the rows of
  its QR, ``(s, shared)`` the columns; the second site's ``(shared, s)``
  form the rows of its LQ; the isometries keep ``k = min(rows, d D)``
  columns (rows), so that every isometry column is a physical direction and
  the edge padding of the new tensors stays zero;
* the fit starts from the rank-D truncated SVD of ``G Theta`` (singular
  values split evenly, each singular pair signed so that the largest-
  magnitude entry of its left vector is positive: the fitted tensors' bond
  gauge then does not depend on the SVD routine) and makes ``n_als`` passes, each solving the normal
  equations for the first reduced tensor, then for the second, with the
  environment symmetrised and ``1e-12 * trace / n`` added to the diagonal;
* after the fit both tensors are scaled to a largest entry of 1 (the state
  changes by a factor only).
"""

import numpy as np

from oracle import blockbp as ob


def bond_order(Lx, Ly):
    """Gate order of one Trotter step: horizontal bonds row by row, then
    vertical bonds column by column; each bond ((x0, y0), (x1, y1))."""
    out = [((x, y), (x + 1, y)) for y in range(Ly) for x in range(Lx - 1)]
    out += [((x, y), (x, y + 1)) for x in range(Lx) for y in range(Ly - 1)]
    return out


def leg_dims(x, y, Lx, Ly, D):
    """True dimensions of the legs (u, l, d, r) of site (x, y) of an open
    lattice: 1 on the lattice edge, D inside."""
    return (1 if y == 0 else D, 1 if x == 0 else D,
            1 if y == Ly - 1 else D, 1 if x == Lx - 1 else D)


def split_pair(Aa, Ab, horizontal, dims_a, dims_b):
    """Reduced tensors of a bond: ``Aa = X_a . R_a`` (QR over the rows
    formed by Aa's legs other than the shared one, at their true
    dimensions dims_a) and ``Ab = L_b . Y_b`` (LQ over the columns formed
    by Ab's other legs, at dims_b).  Returns X_a [rows, k], R_a [k, s, r],
    L_b [r, s, k'], Y_b [k', cols], and the leg orders used to rebuild the
    tensors."""
    d, D = Aa.shape[0], Aa.shape[1]
    # site tensor legs (s, u, l, d, r); shared leg of a: r (horizontal) or
    # d (vertical); of b: l or u
    sa = 4 if horizontal else 3
    sb = 2 if horizontal else 1
    oa = [i for i in (1, 2, 3, 4) if i != sa]
    ob_ = [i for i in (1, 2, 3, 4) if i != sb]
    ta = Aa[(slice(None),) + tuple(slice(0, n) for n in dims_a)]
    tb = Ab[(slice(None),) + tuple(slice(0, n) for n in dims_b)]
    ra = int(np.prod([dims_a[i - 1] for i in oa]))
    cb = int(np.prod([dims_b[i - 1] for i in ob_]))
    Ma = ta.transpose(oa + [0, sa]).reshape(ra, d * D)
    Q, R = np.linalg.qr(Ma)              # Q: rows x k, R: k x (d D)
    k = Q.shape[1]
    Mb = tb.transpose([sb, 0] + ob_).reshape(D * d, cb)
    Qt, Rt = np.linalg.qr(Mb.T)          # Mb = Rt^T Qt^T
    L, Y = Rt.T, Qt.T                    # L: (D d) x k', Y: k' x cols
    kb = Y.shape[0]
    return (Q, R.reshape(k, d, D), L.reshape(D, d, kb), Y, oa, ob_, sa, sb)


def _reduced_site(Xmat, legs, shared, dims, k, dp, D):
    """Site tensor [k, u, l, d, r] (physical dimension dp >= k) of an
    isometry ``Xmat[(legs), k]``, the rows formed by the three legs in
    ``legs`` order at their true dimensions ``dims`` (u, l, d, r), with the
    shared leg at index 0 only and zero padding to D."""
    n = [dims[i - 1] for i in legs]
    E = np.zeros((k, D, D, D, D))        # axes: k, legs[0], legs[1], legs[2], shared
    E[:, :n[0], :n[1], :n[2], 0] = np.moveaxis(Xmat.reshape(n[0], n[1], n[2], k), 3, 0)
    pos = {legs[0]: 1, legs[1]: 2, legs[2]: 3, shared: 4}
    t = np.zeros((dp, D, D, D, D))
    t[:k] = E.transpose([0, pos[1], pos[2], pos[3], pos[4]])
    return t


def bond_environment(bp, A, a, b, Xa, Yb, oa, ob_, sa, sb, k, kb, dims_a, dims_b):
    """Environment N[(k_a,k_b),(k_a',k_b')] of the two reduced tensors: the
    two-site reduced density matrix of the network in which sites a and b
    carry their isometries with the isometry bond as the physical index (the
    shared leg cut to index 0), every other site padded to that physical
    dimension, and the messages of the converged block BP as the region's
    boundary.  Normalised to unit trace (a scale the fit does not see)."""
    d, D = A.shape[1], A.shape[2]
    dp = max(d, k, kb)
    Lx, Ly = bp.Lx, bp.Ly
    M = np.zeros((A.shape[0], dp, D, D, D, D))
    M[:, :d] = A
    ia = a[1] * Lx + a[0]
    ib = b[1] * Lx + b[0]
    M[ia] = _reduced_site(Xa, oa, sa, dims_a, k, dp, D)
    M[ib] = _reduced_site(Yb.T, ob_, sb, dims_b, kb, dp, D)
    env = ob.BlockBP(M, D=D, chi=bp.chi, bx=bp.bx, by=bp.by, Lx=Lx, Ly=Ly,
                     chi_env=bp.chi_env, n_fit=bp.n_fit, seed=bp.seed, d=dp)
    env.msgs = {key: [t.copy() for t in m] for key, m in bp.msgs.items()}
    rho = env.rdm_bond(a[0], a[1], b[0], b[1])          # [(ka,kb), (ka',kb')]
    return rho.reshape(dp, dp, dp, dp)[:k, :kb, :k, :kb].reshape(k * kb, k * kb)


def _solve(Mm, y):
    """Normal equations with the environment symmetrised and a small
    relative diagonal shift."""
    Mm = 0.5 * (Mm + Mm.T)
    n = Mm.shape[0]
    Mm = Mm + 1e-12 * np.trace(Mm) / n * np.eye(n)
    return np.linalg.solve(Mm, y)


def fit_pair(N, Theta, G, D, n_als):
    """Fit ``R'[ka, s, r] L'[r, s', kb]`` (bond D) to ``T = G Theta`` in the
    metric of the environment N[(ka,kb),(ka',kb')] by alternating least
    squares from the truncated SVD of T.  Returns R', L'."""
    k, d, _, kb = Theta.shape
    G4 = G.reshape(d, d, d, d)                           # [s0', s1', s0, s1]
    T = np.einsum("tusv,asvb->atub", G4, Theta)          # [ka, s0', s1', kb]
    U, S, Vt = np.linalg.svd(T.reshape(k * d, d * kb), full_matrices=False)
    r = min(D, S.size)
    # sign of each singular pair: the largest-magnitude entry of u_r positive
    for j in range(r):
        if U[np.argmax(np.abs(U[:, j])), j] < 0:
            U[:, j] = -U[:, j]
            Vt[j] = -Vt[j]
    R = np.zeros((k * d, D))
    Lm = np.zeros((D, d * kb))
    R[:, :r] = U[:, :r] * np.sqrt(S[:r])
    Lm[:r] = np.sqrt(S[:r])[:, None] * Vt[:r]
    R = R.reshape(k, d, D)
    L = Lm.reshape(D, d, kb)
    N4 = N.reshape(k, kb, k, kb)
    for _ in range(n_als):
        # R' with L' fixed: M[(a,s,r),(a',s',r')] = delta_ss' L[r,u,b] N[a,b,a',b'] L[r',u,b']
        Mr = np.einsum("rub,abcd,qud->arcq", L, N4, L)      # [a, r, a', r']
        Mfull = np.einsum("arcq,st->asrctq", Mr, np.eye(d)).reshape(k * d * D, k * d * D)
        y = np.einsum("rub,abcd,csud->asr", L, N4, T).reshape(-1)
        R = _solve(Mfull, y).reshape(k, d, D)
        # L' with R' fixed: M[(r,u,b),(r',u',b')] = delta_uu' R[a,s,r] N[a,b,a',b'] R[a',s,r']
        Ml = np.einsum("asr,abcd,csq->rbqd", R, N4, R)      # [r, b, r', b']
        Mfull = np.einsum("rbqd,uv->rubqvd", Ml, np.eye(d)).reshape(D * d * kb, D * d * kb)
        y = np.einsum("asr,abcd,csud->rub", R, N4, T).reshape(-1)
        L = _solve(Mfull, y).reshape(D, d, kb)
    return R, L


def rebuild(Xa, R, L, Yb, oa, ob_, sa, sb, d, D, dims_a, dims_b):
    """Site tensors [s, u, l, d, r] from the isometries and the fitted
    reduced tensors (zero padding to D on the edge legs), each scaled to a
    largest entry of 1."""
    k, kb = Xa.shape[1], Yb.shape[0]
    na = [dims_a[i - 1] for i in oa]
    nb = [dims_b[i - 1] for i in ob_]
    Ma = (Xa @ R.reshape(k, d * D)).reshape(na + [d, D])    # legs oa, then s, shared
    Mb = (L.reshape(D * d, kb) @ Yb).reshape([D, d] + nb)   # shared, s, legs ob_
    Aa = np.zeros((d, D, D, D, D))
    Ab = np.zeros((d, D, D, D, D))
    ta = _untranspose(Ma, oa + [0, sa])
    tb = _untranspose(Mb, [sb, 0] + ob_)
    Aa[(slice(None),) + tuple(slice(0, n) for n in ta.shape[1:])] = ta
    Ab[(slice(None),) + tuple(slice(0, n) for n in tb.shape[1:])] = tb
    return Aa / np.abs(Aa).max(), Ab / np.abs(Ab).max()


def _untranspose(M, order):
    """Inverse of ``X.transpose(order)``: M's axis i is X's axis order[i]."""
    return np.transpose(M, np.argsort(order))


def ite_step(A, Lx, Ly, D, chi, bx, by, gate, n_als=4, chi_env=None, sweeps=30,
             tol=1e-12, bp=None):
    """One Trotter step of the blockBP update on an open Lx x Ly PEPS:
    converge block BP (at most `sweeps` sweeps or residual < tol), then
    apply the gate to every bond in order with the messages fixed.
    Returns the new tensors and the block-BP state used."""
    A = np.array(A, dtype=np.float64)
    d = A.shape[1]
    if bp is None:
        bp = ob.BlockBP(A, D=D, chi=chi, bx=bx, by=by, Lx=Lx, Ly=Ly, chi_env=chi_env)
    for _ in range(sweeps):
        if bp.sweep() < tol:
            break
    for (a, b) in bond_order(Lx, Ly):
        horizontal = a[1] == b[1]
        ia, ib = a[1] * Lx + a[0], b[1] * Lx + b[0]
        da = leg_dims(a[0], a[1], Lx, Ly, D)
        db = leg_dims(b[0], b[1], Lx, Ly, D)
        Xa, Ra, Lb, Yb, oa, ob_, sa, sb = split_pair(A[ia], A[ib], horizontal, da, db)
        k, kb = Xa.shape[1], Yb.shape[0]
        N = bond_environment(bp, A, a, b, Xa, Yb, oa, ob_, sa, sb, k, kb, da, db)
        Theta = np.einsum("asr,rtb->astb", Ra, Lb)
        R, L = fit_pair(N, Theta, gate, D, n_als)
        A[ia], A[ib] = rebuild(Xa, R, L, Yb, oa, ob_, sa, sb, d, D, da, db)
    return A, bp
