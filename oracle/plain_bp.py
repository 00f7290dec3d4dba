"""Plain BP on the double-layer network of a finite PEPS (test infrastructure).

Blocks of a single site reduce block BP to the BP contraction of Alkabetz and
Arad (Sec. II, paragraph on blocks of size 1): each message is a vector over a
fused double-layer bond (a D x D matrix), updated from the three other
incoming messages of its site and normalised to unit 2-norm.  Written
independently of ``blockbp`` (no orientation frames, no fits) so that it pins
the block code's leg and orientation bookkeeping.
"""

import numpy as np

SIDES = ("U", "L", "D", "R")  # leg order of E[u, l, d, r]
NEIGH = {"U": (0, -1), "L": (-1, 0), "D": (0, 1), "R": (1, 0)}
OPP = {"U": "D", "D": "U", "L": "R", "R": "L"}


def _double(A, Aket):
    D = A.shape[1]
    return np.einsum("suldr,sULDR->uUlLdDrR", Aket, A).reshape(
        D * D, D * D, D * D, D * D)


class PlainBP:
    def __init__(self, A, Lx, Ly):
        self.A, self.Lx, self.Ly = A, Lx, Ly
        D = A.shape[2]
        self.q = D * D
        self.E = [_double(a, a) for a in A]
        eye = (np.eye(D) / np.sqrt(D)).reshape(-1)
        self.m = {}
        for y in range(Ly):
            for x in range(Lx):
                for s in SIDES:
                    if self._inside(x, y, s):
                        self.m[(x, y, s)] = eye.copy()

    def _inside(self, x, y, s):
        dx, dy = NEIGH[s]
        return 0 <= x + dx < self.Lx and 0 <= y + dy < self.Ly

    def incoming(self, x, y, s, m=None):
        """Vector arriving at (x, y) on leg ``s``; e_0 on an open edge."""
        m = self.m if m is None else m
        if not self._inside(x, y, s):
            v = np.zeros(self.q)
            v[0] = 1.0
            return v
        dx, dy = NEIGH[s]
        return m[(x + dx, y + dy, OPP[s])]

    def sweep(self):
        new = {}
        for (x, y, s), _ in self.m.items():
            E = self.E[y * self.Lx + x]
            vecs = [self.incoming(x, y, t) for t in SIDES]
            k = SIDES.index(s)
            t = E
            # contract every leg but k, highest axis first
            for ax in range(3, -1, -1):
                if ax != k:
                    t = np.tensordot(t, vecs[ax], axes=([ax], [0]))
            new[(x, y, s)] = t / np.linalg.norm(t)
        self.m = new

    def site_value(self, x, y, op=None):
        a = self.A[y * self.Lx + x]
        ak = a if op is None else np.einsum("ts,suldr->tuldr", op, a)
        t = _double(a, ak)
        for ax in range(3, -1, -1):
            t = np.tensordot(t, self.incoming(x, y, SIDES[ax]), axes=([ax], [0]))
        return float(t)

    def expect_site(self, x, y, op):
        return self.site_value(x, y, op) / self.site_value(x, y)
