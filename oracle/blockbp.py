"""FP64 oracle for block belief propagation on 2D PEPS (Guo, Poletti, Arad,
"Block belief propagation algorithm for two-dimensional tensor networks").

TEST INFRASTRUCTURE.  Plain NumPy, slow and direct: einsum for every
contraction, ``numpy.linalg.qr`` (LAPACK Householder) for QR/LQ.  Only the
tests, the smoke check and the benchmark's CPU baseline use it.  It shares no
code with the GPU library.

What it computes, by section of the paper
-----------------------------------------
* Double layer (Sec. II, Fig. 1(a,b)): ``E = sum_s A[s] (x) A[s]``, each fused
  leg of dimension D^2 with index ``q = k*D + k'`` (ket-major).  Tensors are
  real, so the bra needs no conjugation.
* Block partition (Sec. II, Fig. 1(c)) and the message equation, Eq. (1):
  ``m_{A->B} = Tr(T_A prod_{A' in N_A \\ B} m_{A'->A})``, iterated
  synchronously: every message of sweep l+1 uses only sweep-l messages.
* Message contraction (App. A, Fig. 1(d)): the block is contracted with its
  three other incoming messages column by column from the side opposite the
  receiver, keeping a bond of at most chi after every column.
* Each column absorption is an MPO x MPS product done by the variational fit of
  App. A: minimise ``||Y - O X||^2`` (Eq. distance) with DMRG-like sweeps, the
  local update Eq. (update) with left/right environments built recursively
  from ``A_1 = B_{L+1} = 1``, QR on left-to-right steps and LQ on
  right-to-left steps, Q becoming the new site tensor.
* Finite-lattice edges carry trivial messages (App. A; Sec. II on open
  boundaries embedded with bond dimension 1).
* Infinite lattices: one block that sends messages to and receives messages
  from its own copies (Sec. II, last paragraphs on iPEPS).
* Residual: distance between normalised messages of consecutive sweeps (Sec.
  II convergence test; App. A mean-square error).
* Observables from the converged messages (Sec. II; App. A second paragraph;
  App. B boundary-MPS procedure with trivial corner tensors): boundary MPSs are
  absorbed from the two sides at bond chi_env, the last line is contracted
  exactly with and without the operator.

Readings where the paper is silent (each also listed in the design notes):
synchronous updates without damping; identity product initial messages;
2-norm message normalisation, sign free; residual = mean over messages of the
squared sign-aligned distance ``max(0, 2 - 2|<m_new, m_old>|)``; fixed number of
fit sweeps ``n_fit``; fit initial state = the previous sweep's result for the
same slot when its shapes agree, otherwise a counter-based uniform random MPS
(SplitMix64) right-canonicalised by LQ; bond caps ``min(chi, bX_j*w_j)`` made
consistent with the physical dimensions; messages are open MPSs with
dimension-1 end bonds; a bond crossing two blocks is evaluated on the union of
the two blocks; a vertical bond is evaluated on a column (the region seen
rotated by 90 degrees); log-norm from the block Bethe formula
``sum_A log|Z_A| - sum_edges log|Z_AB|``.
"""

import math

import numpy as np

DIRS = ("L", "R", "U", "D")
OPP = {"L": "R", "R": "L", "U": "D", "D": "U"}
STEP = {"L": (-1, 0), "R": (1, 0), "U": (0, -1), "D": (0, 1)}
DIR_INDEX = {"L": 0, "R": 1, "U": 2, "D": 3}

# ---------------------------------------------------------------------------
# Counter-based uniform numbers: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014).
# ---------------------------------------------------------------------------
_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_C1 = np.uint64(0xBF58476D1CE4E5B9)
_C2 = np.uint64(0x94D049BB133111EB)


def _splitmix(x):
    """SplitMix64 output function applied to state ``x`` (numpy uint64 arrays
    wrap modulo 2^64)."""
    with np.errstate(over="ignore"):
        z = x + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _C1
        z = (z ^ (z >> np.uint64(27))) * _C2
        return z ^ (z >> np.uint64(31))


def counter_uniform(seed, slot, site, n):
    """``n`` numbers ``2*(h >> 11)*2^-53 - 1`` in [-1, 1) with
    ``h = sm(sm(sm(sm(seed) ^ slot) ^ site) ^ i)`` for ``i = 0..n-1``.
    Every value is exact in FP64."""
    h = _splitmix(np.uint64(seed))
    h = _splitmix(h ^ np.uint64(slot))
    h = _splitmix(h ^ np.uint64(site))
    idx = np.arange(n, dtype=np.uint64)
    v = _splitmix(h ^ idx)
    return (v >> np.uint64(11)).astype(np.float64) * (2.0 ** -52) - 1.0


def slot_message(e, col):
    return (1 << 40) | (e << 8) | col


def slot_region(kind, bi, bj, orient, col):
    return ((2 << 40) | (kind << 36) | (bj << 24) | (bi << 12)
            | (DIR_INDEX[orient] << 8) | col)


# ---------------------------------------------------------------------------
# Double layer and small MPS utilities
# ---------------------------------------------------------------------------
def double_layer(A, Aket=None):
    """``E[(u u'),(l l'),(d d'),(r r')] = sum_s Aket[s,u,l,d,r] A[s,u',l',d',r']``
    (Sec. II, Fig. 1(a,b)); ``Aket = O @ A`` inserts a one-site operator."""
    if Aket is None:
        Aket = A
    D = A.shape[1]
    E = np.einsum("suldr,sULDR->uUlLdDrR", Aket, A)
    return E.reshape(D * D, D * D, D * D, D * D)


def single_layer_bra(A):
    """Bra tensor of a single-layer network (Sec. V classical Ising; App. A
    single-layer messages): every virtual leg at index 0 for each value of
    the split index s, so that the double layer ``sum_s A[s] (x) bra[s]``
    is the single-layer tensor ``T = sum_s A[s]`` placed at the fused
    indices (k, 0), and a one-site operator O inserts
    ``sum_s (sum_s' O[s', s]) A[s]`` (for a diagonal O: the impurity
    tensor ``sum_s O[s, s] A[s]``)."""
    B = np.zeros_like(A)
    B[:, 0, 0, 0, 0] = 1.0
    return B


def apply_op(op, A):
    """Ket tensor with a one-site operator applied: ``sum_s op[s', s] A[s]``."""
    return np.einsum("ts,suldr->tuldr", op, A)


def trivial_mps(n, D):
    """Trivial boundary message: every site selects fused index 0, bonds 1."""
    t = np.zeros((1, D * D, 1))
    t[0, 0, 0] = 1.0
    return [t.copy() for _ in range(n)]


def identity_mps(n, D):
    """Identity product MPDO, ``m[q=(k,k')] = delta_{kk'} / sqrt(D)`` per site."""
    t = (np.eye(D) / math.sqrt(D)).reshape(1, D * D, 1)
    return [t.copy() for _ in range(n)]


def random_mpdo(n, D, seed, e):
    """Random product MPDO (App. A's random initial message, here with the
    counter-based uniform values instead of normal ones so that every
    implementation draws the same numbers): site i is ``R R^T`` for the D x D
    matrix R of ``counter_uniform(seed, 2^41 + e, i, D*D)``, scaled to unit
    Frobenius norm; positive semidefinite, bonds 1."""
    out = []
    for i in range(n):
        R = counter_uniform(seed, (1 << 41) + e, i, D * D).reshape(D, D)
        M = R @ R.T
        out.append((M / np.linalg.norm(M)).reshape(1, D * D, 1))
    return out


def mps_reverse(m):
    """Reverse the site order; each site's two bond legs swap."""
    return [t.transpose(2, 1, 0).copy() for t in reversed(m)]


def mps_overlap(a, b):
    """``<a|b>`` for two open MPSs with equal physical dimensions."""
    env = np.ones((1, 1))
    for ta, tb in zip(a, b):
        env = np.einsum("ab,apc,bpd->cd", env, ta, tb)
    return float(env[0, 0])


def mps_dense(m):
    """Dense vector of an open MPS (small cases only)."""
    v = m[0]
    for t in m[1:]:
        v = np.tensordot(v, t, axes=([v.ndim - 1], [0]))
    return v.reshape(-1)


# ---------------------------------------------------------------------------
# MPO x MPS variational fit (App. A)
# ---------------------------------------------------------------------------
# Pairwise contraction orders, given explicitly: einsum's automatic search
# refuses intermediates larger than the inputs and would fall back to the
# naive all-index loop.
_PATH_ENV_L = ["einsum_path", (0, 3), (1, 2), (0, 1)]
_PATH_ENV_R = ["einsum_path", (0, 3), (1, 2), (0, 1)]
_PATH_LOCAL = ["einsum_path", (0, 2), (0, 2), (0, 1)]


def env_left(Le, Y, O, X):
    """Left environment recursion of App. A:
    ``A_{l+1}[y',w',x'] = sum A_l[y,w,x] Y[y,p,y'] O[w,p,q,w'] X[x,q,x']``."""
    return np.einsum("ywx,ypu,wpqv,xqz->uvz", Le, Y, O, X,
                     optimize=_PATH_ENV_L)


def env_right(Re, Y, O, X):
    """Right environment recursion of App. A:
    ``B_l[y,w,x] = sum B_{l+1}[y',w',x'] Y[y,p,y'] O[w,p,q,w'] X[x,q,x']``."""
    return np.einsum("uvz,ypu,wpqv,xqz->ywx", Re, Y, O, X,
                     optimize=_PATH_ENV_R)


def local_update(Le, O, X, Re):
    """Eq. (update): ``Yt[y,p,y'] = sum A[y,w,x] O[w,p,q,w'] B[y',w',x'] X[x,q,x']``."""
    return np.einsum("ywx,wpqv,xqz,uvz->ypu", Le, O, X, Re,
                     optimize=_PATH_LOCAL)


def bond_caps(O, X, chi):
    """Bond dimensions of Y.  ``b_j = min(chi, bX_j * w_j)``: no bond exceeds
    what O X can fill; then made consistent with the physical dimensions so
    that every QR panel is tall and every LQ panel is wide."""
    N = len(X)
    p = [O[j].shape[1] for j in range(N)]
    b = [min(chi, X[j].shape[2] * O[j].shape[3]) for j in range(N - 1)]
    for j in range(N - 1):
        left = b[j - 1] if j > 0 else 1
        b[j] = min(b[j], left * p[j])
    for j in range(N - 1, 0, -1):
        right = b[j] if j < N - 1 else 1
        b[j - 1] = min(b[j - 1], p[j] * right)
    return p, b


def _lq(M):
    """LQ of a wide matrix through the QR of its transpose."""
    q, r = np.linalg.qr(M.T)
    return r.T, q.T


def fit(O, X, chi, n_fit, seed, slot, Yinit=None):
    """Variational fit ``Y ~ O X`` (App. A).

    Returns ``(Y, nu)``: ``Y[1:]`` right-orthonormal, ``Y[0]`` the final
    centre ``Yt_0`` (norm ``nu``), so ``||Y|| = nu``.  Start: ``Yinit`` if its
    shapes agree with the caps, else a counter-based uniform random MPS
    brought to right-canonical form by LQ.  Then ``n_fit`` full sweeps
    (left-to-right with QR, right-to-left with LQ); no early exit.
    """
    N = len(X)
    p, b = bond_caps(O, X, chi)
    shapes = [((b[j - 1] if j > 0 else 1), p[j], (b[j] if j < N - 1 else 1))
              for j in range(N)]
    if Yinit is not None and all(t.shape == s for t, s in zip(Yinit, shapes)):
        Y = [t.copy() for t in Yinit]
    else:
        Y = [counter_uniform(seed, slot, j, int(np.prod(s))).reshape(s)
             for j, s in enumerate(shapes)]
        for j in range(N - 1, 0, -1):
            bl, pj, br = Y[j].shape
            L, Q = _lq(Y[j].reshape(bl, pj * br))
            Y[j] = Q.reshape(bl, pj, br)
            Y[j - 1] = np.einsum("apb,bc->apc", Y[j - 1], L)
    one = np.ones((1, 1, 1))
    Le = [None] * N
    Re = [None] * N
    Le[0] = one
    Re[N - 1] = one
    for j in range(N - 1, 0, -1):
        Re[j - 1] = env_right(Re[j], Y[j], O[j], X[j])
    for _ in range(n_fit):
        for j in range(0, N - 1):
            Yt = local_update(Le[j], O[j], X[j], Re[j])
            bl, pj, br = Yt.shape
            Q, _ = np.linalg.qr(Yt.reshape(bl * pj, br))
            Y[j] = Q.reshape(bl, pj, br)
            Le[j + 1] = env_left(Le[j], Y[j], O[j], X[j])
        for j in range(N - 1, 0, -1):
            Yt = local_update(Le[j], O[j], X[j], Re[j])
            bl, pj, br = Yt.shape
            _, Q = _lq(Yt.reshape(bl, pj * br))
            Y[j] = Q.reshape(bl, pj, br)
            Re[j - 1] = env_right(Re[j], Y[j], O[j], X[j])
    Y[0] = local_update(Le[0], O[0], X[0], Re[0])
    nu = float(np.linalg.norm(Y[0]))
    return Y, nu


# ---------------------------------------------------------------------------
# Regions, orientation and column absorption (App. A, Fig. 1(d))
# ---------------------------------------------------------------------------
# Leg permutation taking A[s,u,l,d,r] to the frame in which the output side
# is on the left: "L" identity, "R" half turn, "U" quarter turn
# counter-clockwise, "D" quarter turn clockwise.
ROT_PERM = {"L": (0, 1, 2, 3, 4), "R": (0, 3, 4, 1, 2),
            "U": (0, 4, 1, 2, 3), "D": (0, 2, 3, 4, 1)}
OUT_REVERSED = {"L": False, "R": True, "U": True, "D": False}


class Region:
    """A rectangle of sites with its four incoming boundary MPSs.

    ``A[y][x]`` site tensors (H rows, W columns); ``T``/``B`` top/bottom
    messages with W sites ordered left to right, ``L``/``R`` left/right
    messages with H sites ordered top to bottom.
    """

    def __init__(self, A, T, B, L, R):
        self.A, self.T, self.B, self.L, self.R = A, T, B, L, R
        self.H = len(A)
        self.W = len(A[0])


def canonical(reg, orient):
    """Rotate a region so that side ``orient`` is on the left.  Returns the
    rotated grid and the incoming top/right/bottom MPSs in the rotated frame."""
    H, W = reg.H, reg.W
    perm = ROT_PERM[orient]
    if orient == "L":
        grid = [[reg.A[y][x] for x in range(W)] for y in range(H)]
        MT, MR, MB = reg.T, reg.R, reg.B
    elif orient == "R":
        grid = [[reg.A[H - 1 - y][W - 1 - x] for x in range(W)] for y in range(H)]
        MT, MR, MB = mps_reverse(reg.B), mps_reverse(reg.L), mps_reverse(reg.T)
    elif orient == "U":
        grid = [[reg.A[x][W - 1 - y] for x in range(H)] for y in range(W)]
        MT, MR, MB = reg.R, mps_reverse(reg.B), reg.L
    else:  # "D"
        grid = [[reg.A[H - 1 - x][y] for x in range(H)] for y in range(W)]
        MT, MR, MB = mps_reverse(reg.L), reg.T, mps_reverse(reg.R)
    grid = [[t.transpose(perm) for t in row] for row in grid]
    return grid, MT, MR, MB


def column_mpo(Egrid, MT, MB, c):
    """MPO of column c, sites ``[MT[c], E[0,c], ..., E[H-1,c], MB[c]]``, each
    as ``O[w_up, p_out(left), p_in(right), w_down]``."""
    O = [MT[c].transpose(0, 2, 1)[None, ...]]
    for row in Egrid:
        O.append(row[c].transpose(0, 1, 3, 2))
    O.append(MB[c].transpose(1, 0, 2)[..., None])
    return O


def absorb(grid, MT, MR, MB, chi, n_fit, seed, slot_fn, ncols=None,
           warm=None, keep=False, bra=None):
    """Contract canonical columns right to left into a boundary MPS.

    The boundary starts as ``[1, MR..., 1]`` (trivial corners) and after each
    column is replaced by ``fit(column MPO, boundary)`` normalised to unit
    norm, the logarithm of the norm being accumulated.  Returns the final
    boundary, its log-scale, the list of ``(boundary, logscale)`` after
    0, 1, ... columns when ``keep``, and the per-column fit results.
    ``bra`` maps a site tensor to its bra layer (default: the tensor itself)."""
    H, W = len(grid), len(grid[0])
    Egrid = [[double_layer(bra(t) if bra else t, t) for t in row] for row in grid]
    one = np.ones((1, 1, 1))
    X = [one] + list(MR) + [one]
    log_scale = 0.0
    stack = [(X, 0.0)] if keep else None
    ncols = W if ncols is None else ncols
    fits = {}
    for c in range(W - 1, W - 1 - ncols, -1):
        O = column_mpo(Egrid, MT, MB, c)
        Y, nu = fit(O, X, chi, n_fit, seed, slot_fn(c),
                    None if warm is None else warm.get(c))
        if not (nu > 0.0 and np.isfinite(nu)):
            raise FloatingPointError("zero or non-finite boundary norm")
        Y[0] = Y[0] / nu
        log_scale += math.log(nu)
        fits[c] = [t.copy() for t in Y]
        X = Y
        if keep:
            stack.append((X, log_scale))
    return X, log_scale, stack, fits


def extract_message(Y):
    """Contract the two dimension-1 end sites of the final boundary into their
    neighbours, giving an L-site message with dimension-1 end bonds."""
    N = len(Y)
    m = [t.copy() for t in Y[1:N - 1]]
    m[0] = np.einsum("abc,cpd->apd", Y[0], m[0]).reshape(1, *m[0].shape[1:])
    m[-1] = np.einsum("apb,bcd->apd", m[-1], Y[N - 1])
    return m


# ---------------------------------------------------------------------------
# Lattice, partition and the sweep (Sec. II, Eq. (1))
# ---------------------------------------------------------------------------
class BlockBP:
    """Block BP state for a finite open lattice or an infinite one.

    Finite: ``A`` has ``Ly*Lx`` tensors.  Lattices that are not multiples of
    the block are padded with trivial sites (``A[0,0,0,0,0] = 1``), which
    leaves the network's value unchanged.
    Infinite: ``A`` has ``ucy*ucx`` unit-cell tensors; the block must be a
    multiple of the cell and is the only block.
    """

    def __init__(self, A, D, chi, bx, by, Lx=0, Ly=0, infinite=False,
                 ucx=1, ucy=1, chi_env=None, n_fit=2, seed=0, d=2, shift=(0, 0),
                 single_layer=False, init=0):
        self.D, self.chi, self.bx, self.by = D, chi, bx, by
        # single-layer network: the tensors' sum over s is the network
        # tensor, the bra layer a fixed index-0 tensor
        self.bra = single_layer_bra if single_layer else None
        self.infinite = infinite
        self.d = d
        self.chi_env = (2 * D * D + 10) if chi_env is None else chi_env
        self.n_fit, self.seed = n_fit, seed
        A = np.asarray(A, dtype=np.float64)
        if infinite:
            if bx % ucx or by % ucy:
                raise ValueError("block must be a multiple of the unit cell")
            self.ucx, self.ucy = ucx, ucy
            self.gx = self.gy = 1
            self.site = lambda x, y: A[(y % ucy) * ucx + (x % ucx)]
        else:
            # shifted partition (Sec. II: partitions that differ by a shift
            # of the lattice): sx trivial columns on the left and sy trivial
            # rows on top, the same as shifting an OBC lattice embedded in a
            # periodic one with dimension-1 bonds at its edges
            sx, sy = shift
            if not (0 <= sx < bx and 0 <= sy < by):
                raise ValueError("shift must lie inside one block")
            self.Lx, self.Ly = Lx, Ly
            self.sx, self.sy = sx, sy
            self.gx = -(-(Lx + sx) // bx)
            self.gy = -(-(Ly + sy) // by)
            triv = np.zeros((d, D, D, D, D))
            triv[0, 0, 0, 0, 0] = 1.0

            def site(x, y, A=A):
                x, y = x - sx, y - sy
                if 0 <= x < Lx and 0 <= y < Ly:
                    return A[y * Lx + x]
                return triv
            self.site = site
        self.msgs = {}
        self.order = []
        for bj in range(self.gy):
            for bi in range(self.gx):
                for dr in DIRS:
                    if self.neighbour(bi, bj, dr) is not None:
                        self.order.append((bi, bj, dr))
        for e, (bi, bj, dr) in enumerate(self.order):
            n = by if dr in ("L", "R") else bx
            self.msgs[(bi, bj, dr)] = (identity_mps(n, D) if init == 0
                                       else random_mpdo(n, D, seed, e))
        self.warm = {k: {} for k in self.order}
        self.residuals = []
        self._cache = {}

    # -- block graph ---------------------------------------------------------
    def neighbour(self, bi, bj, dr):
        if self.infinite:
            return (bi, bj)
        dx, dy = STEP[dr]
        ni, nj = bi + dx, bj + dy
        if 0 <= ni < self.gx and 0 <= nj < self.gy:
            return (ni, nj)
        return None

    def incoming(self, bi, bj, side, msgs=None):
        """Message arriving at block (bi,bj) from its neighbour on ``side``:
        that neighbour's message in the opposite direction, or the trivial
        message on a finite lattice edge."""
        msgs = self.msgs if msgs is None else msgs
        nb = self.neighbour(bi, bj, side)
        n = self.by if side in ("L", "R") else self.bx
        if nb is None:
            return trivial_mps(n, self.D)
        return msgs[(nb[0], nb[1], OPP[side])]

    def block_grid(self, bi, bj):
        return [[self.site(bi * self.bx + x, bj * self.by + y)
                 for x in range(self.bx)] for y in range(self.by)]

    def block_region(self, bi, bj, msgs=None):
        return Region(self.block_grid(bi, bj),
                      self.incoming(bi, bj, "U", msgs),
                      self.incoming(bi, bj, "D", msgs),
                      self.incoming(bi, bj, "L", msgs),
                      self.incoming(bi, bj, "R", msgs))

    # -- Eq. (1) ---------------------------------------------------------------
    def update_message(self, e_index, key, msgs):
        bi, bj, dr = key
        grid, MT, MR, MB = canonical(self.block_region(bi, bj, msgs), dr)
        Y, _, _, fits = absorb(grid, MT, MR, MB, self.chi, self.n_fit,
                               self.seed,
                               lambda c: slot_message(e_index, c),
                               warm=self.warm[key], bra=self.bra)
        self.warm[key] = fits
        m = extract_message(Y)
        return mps_reverse(m) if OUT_REVERSED[dr] else m

    def sweep(self, n=1):
        """``n`` synchronous sweeps; returns the last sweep's residual, the mean
        over messages of ``max(0, 2 - 2|<m_new, m_old>|)``."""
        res = None
        for _ in range(n):
            old = self.msgs
            new = {}
            for e, key in enumerate(self.order):
                new[key] = self.update_message(e, key, old)
            deltas = [max(0.0, 2.0 - 2.0 * abs(mps_overlap(new[k], old[k])))
                      for k in self.order]
            res = float(np.mean(deltas)) if deltas else 0.0
            self.msgs = new
            self.residuals.append(res)
            self._cache = {}
        return res

    # -- observables (Sec. II; App. A; App. B) ---------------------------------
    def _region(self, kind, bi, bj):
        if kind == 0:
            return self.block_region(bi, bj)
        a = self.block_region(bi, bj)
        if kind == 1:  # horizontal union of (bi,bj) and its right neighbour
            ni, nj = self.neighbour(bi, bj, "R")
            b = self.block_region(ni, nj)
            grid = [ra + rb for ra, rb in zip(a.A, b.A)]
            return Region(grid, a.T + b.T, a.B + b.B, a.L, b.R)
        ni, nj = self.neighbour(bi, bj, "D")  # kind 2: vertical union
        b = self.block_region(ni, nj)
        return Region(a.A + b.A, a.T, b.B, a.L + b.L, a.R + b.R)

    def _stack(self, kind, bi, bj, orient):
        """Boundaries after absorbing 0..n-1 lines of the region from the side
        opposite ``orient`` at bond chi_env."""
        key = (kind, bi, bj, orient)
        if key not in self._cache:
            reg = self._region(kind, bi, bj)
            grid, MT, MR, MB = canonical(reg, orient)
            W = len(grid[0])
            _, _, stack, _ = absorb(
                grid, MT, MR, MB, self.chi_env, self.n_fit, self.seed,
                lambda c: slot_region(kind, bi, bj, orient, c),
                ncols=W - 1, keep=True, bra=self.bra)
            self._cache[key] = (reg, stack)
        return self._cache[key]

    def _line(self, kind, bi, bj, axis, k):
        """Top/bottom (axis 'row') or left/right (axis 'col') boundaries of
        line k, the line's sites, its end messages and the boundaries' log
        scale."""
        if axis == "row":
            reg, sd = self._stack(kind, bi, bj, "D")
            _, su = self._stack(kind, bi, bj, "U")
            up, lu = sd[k]
            dn, ld = su[reg.H - 1 - k]
            dn = mps_reverse(dn)
            sites = reg.A[k]
            ends = (reg.L[k], reg.R[k])
            # line MPO legs: O[w_left, p_up, p_down, w_right]
            legs = (2, 1, 3, 4)
        else:
            reg, sr = self._stack(kind, bi, bj, "R")
            _, sl = self._stack(kind, bi, bj, "L")
            up, lu = sr[k]
            up = mps_reverse(up)
            dn, ld = sl[reg.W - 1 - k]
            sites = [reg.A[y][k] for y in range(reg.H)]
            ends = (reg.T[k], reg.B[k])
            # column MPO legs: O[w_up, p_left, p_right, w_down]
            legs = (1, 2, 4, 3)
        return up, dn, sites, ends, legs, lu + ld

    def _contract_line(self, up, dn, sites, ends, legs, ops):
        """Exact contraction of boundary ``up``, the line and boundary ``dn``.
        ``ops`` maps a line position to a one-site operator, or a pair
        ``(i, i+1)`` to a two-site operator ``[(s0',s1'),(s0,s1)]``."""
        first, last = ends
        env = np.ones((1, 1, 1))
        # end message site m[a_up, q, a_down] as O[1, a_up, a_down, q]
        env = env_left(env, up[0], first.transpose(0, 2, 1)[None, ...], dn[0])
        pair = next((k for k in ops if isinstance(k, tuple)), None)
        n = len(sites)
        i = 0
        while i < n:
            A = sites[i].transpose((0,) + legs)
            B = self.bra(A) if self.bra else A
            if pair is not None and i == pair[0]:
                A1 = sites[i + 1].transpose((0,) + legs)
                B1 = self.bra(A1) if self.bra else A1
                op2 = ops[pair].reshape(self.d, self.d, self.d, self.d)
                env = self._pair(env, up[i + 1], up[i + 2], dn[i + 1],
                                 dn[i + 2], op2, A, A1, B, B1)
                i += 2
                continue
            Ak = apply_op(ops[i], A) if i in ops else A
            E = double_layer(B, Ak)  # O[w_left, p_up, p_down, w_right]
            env = env_left(env, up[i + 1], E, dn[i + 1])
            i += 1
        env = env_left(env, up[n + 1], last.transpose(1, 0, 2)[..., None],
                       dn[n + 1])
        return float(env[0, 0, 0])

    def _pair(self, env, y0, y1, x0, x1, op2, A0, A1, B0, B1):
        """Environment step over two neighbouring sites with a two-site
        operator ``op2[s0', s1', s0, s1]`` between their ket (``s``) and bra
        (``s'``) layers.  ``A0``, ``A1`` (ket) and ``B0``, ``B1`` (bra) are
        in line-MPO leg order ``[s, w_left, p_up, p_down, w_right]``."""
        Dk = A0.shape[1]
        e = env.reshape(env.shape[0], Dk, Dk, env.shape[2])
        y0 = y0.reshape(y0.shape[0], Dk, Dk, y0.shape[2])
        y1 = y1.reshape(y1.shape[0], Dk, Dk, y1.shape[2])
        x0 = x0.reshape(x0.shape[0], Dk, Dk, x0.shape[2])
        x1 = x1.reshape(x1.shape[0], Dk, Dk, x1.shape[2])
        # out[d,w,y,g] = sum e[a,i,j,b] y0[a,k,l,c] y1[c,m,n,d] x0[b,o,p,e]
        #   x1[e,q,r,g] op2[t,u,s,v] A0[s,i,k,o,h] A1[v,h,m,q,w]
        #   B0[t,j,l,p,x] B1[u,x,n,r,y], one pair at a time
        t = np.einsum("aijb,aklc->ijbklc", e, y0, optimize=True)
        t = np.einsum("ijbklc,sikoh->jblcsoh", t, A0, optimize=True)
        t = np.einsum("jblcsoh,tjlpx->bcsohtpx", t, B0, optimize=True)
        t = np.einsum("bcsohtpx,bope->cshtxe", t, x0, optimize=True)
        t = np.einsum("cshtxe,tusv->chxeuv", t, op2, optimize=True)
        t = np.einsum("chxeuv,cmnd->hxeuvmnd", t, y1, optimize=True)
        t = np.einsum("hxeuvmnd,vhmqw->xeundqw", t, A1, optimize=True)
        t = np.einsum("xeundqw,uxnry->edqwry", t, B1, optimize=True)
        out = np.einsum("edqwry,eqrg->dwyg", t, x1, optimize=True)
        return out.reshape(out.shape[0], Dk * Dk, out.shape[3])

    def _where(self, x, y):
        """Region-local data of site (x, y): block indices and position."""
        if self.infinite:
            ox = (self.bx - self.ucx) // 2
            oy = (self.by - self.ucy) // 2
            x = ox + (x - ox) % self.ucx
            y = oy + (y - oy) % self.ucy
        else:
            x, y = x + self.sx, y + self.sy
        return x // self.bx, y // self.by, x % self.bx, y % self.by

    def expect_site(self, x, y, op):
        bi, bj, lx, ly = self._where(x, y)
        line = self._line(0, bi, bj, "row", ly)
        up, dn, sites, ends, legs, _ = line
        num = self._contract_line(up, dn, sites, ends, legs, {lx: op})
        den = self._contract_line(up, dn, sites, ends, legs, {})
        return num / den

    def expect_bond(self, x0, y0, x1, y1, op2):
        """Nearest-neighbour bond; ``op2[(s0',s1'),(s0,s1)]`` with site
        (x0,y0) the major index.  (x1,y1) must be (x0+1,y0) or (x0,y0+1)."""
        if (x1, y1) == (x0 + 1, y0):
            horizontal = True
        elif (x1, y1) == (x0, y0 + 1):
            horizontal = False
        else:
            raise ValueError("bond must point right or down")
        bi, bj, lx, ly = self._where(x0, y0)
        if horizontal:
            kind = 0 if lx + 1 < self.bx else 1
            line = self._line(kind, bi, bj, "row", ly)
            pos = lx
        else:
            kind = 0 if ly + 1 < self.by else 2
            line = self._line(kind, bi, bj, "col", lx)
            pos = ly
        up, dn, sites, ends, legs, _ = line
        num = self._contract_line(up, dn, sites, ends, legs,
                                  {(pos, pos + 1): op2})
        den = self._contract_line(up, dn, sites, ends, legs, {})
        return num / den

    def rdm_site(self, x, y):
        """One-site reduced density matrix ``rho[s, s']`` with
        ``<O> = Tr(rho O)``: entry (s, s') is the expectation of the matrix
        unit |s'><s|."""
        d = self.d
        rho = np.zeros((d, d))
        for s in range(d):
            for sp in range(d):
                unit = np.zeros((d, d))
                unit[sp, s] = 1.0
                rho[s, sp] = self.expect_site(x, y, unit)
        return rho

    def rdm_bond(self, x0, y0, x1, y1):
        """Two-site reduced density matrix ``rho[(s0,s1), (s0',s1')]`` of a
        nearest-neighbour bond, (x0, y0) the major index."""
        d2 = self.d * self.d
        rho = np.zeros((d2, d2))
        for a in range(d2):
            for b in range(d2):
                unit = np.zeros((d2, d2))
                unit[b, a] = 1.0
                rho[a, b] = self.expect_bond(x0, y0, x1, y1, unit)
        return rho

    def log_norm(self):
        """Block Bethe formula: ``sum_A log|Z_A| - sum_edges log|Z_AB|``, with
        ``Z_A`` the contraction of block A with its four incoming messages
        (line 0, lower boundary from the chi_env stack) and
        ``Z_AB = <m_{A->B}, m_{B->A}>``.  Returns ``(log|Z|, sign)``."""
        total, sign = 0.0, 1.0
        for bj in range(self.gy):
            for bi in range(self.gx):
                up, dn, sites, ends, legs, ls = self._line(0, bi, bj, "row", 0)
                z = self._contract_line(up, dn, sites, ends, legs, {})
                total += math.log(abs(z)) + ls
                sign *= math.copysign(1.0, z)
        for (bi, bj, dr) in self.order:
            if dr not in ("R", "D"):
                continue
            ni, nj = self.neighbour(bi, bj, dr)
            zab = mps_overlap(self.msgs[(bi, bj, dr)],
                              self.msgs[(ni, nj, OPP[dr])])
            total -= math.log(abs(zab))
            sign *= math.copysign(1.0, zab)
        return total, sign


# ---------------------------------------------------------------------------
# Shifted partitions and trace distances (Sec. II; App. C)
# ---------------------------------------------------------------------------
def trace_distance(rho, sigma):
    """``D(rho, sigma) = Tr|rho - sigma| / 2`` with ``|Z| = sqrt(Z^T Z)``
    (App. C): half the sum of the singular values of the difference."""
    return 0.5 * float(np.sum(np.linalg.svd(np.asarray(rho) - np.asarray(sigma),
                                            compute_uv=False)))


def centre_depth(b, s, x0, x1):
    """How deep the coordinates x0..x1 (x1 = x0 or x0 + 1) lie inside their
    block of size b along one axis when the partition is shifted by s: the
    distance to the nearer block edge, or -1 when they fall in two blocks."""
    u0, u1 = (x0 + s) % b, (x1 + s) % b
    if (x0 + s) // b != (x1 + s) // b:
        return -1
    return min(u0, b - 1 - u1)


def best_shift(bx, by, shifts, x0, y0, x1, y1):
    """The partition shift among ``shifts`` that puts a site (x1, y1 =
    x0, y0) or a bond deepest inside one block: the observable is then
    taken at the centre of its block (Sec. II).  Ties go to the first."""
    best, depth = None, -2
    for (sx, sy) in shifts:
        dep = min(centre_depth(bx, sx, x0, x1), centre_depth(by, sy, y0, y1))
        if dep > depth:
            best, depth = (sx, sy), dep
    return best, depth
