"""Random spin-adapted (SU(2) x U(1)) matrix product states in mixed canonical form.

Conventions (the data layout both the library and its checker read; this
module draws the numbers, it does not compute with them):

* Orbitals 0..n-1 in chain order.  Local multiplets sigma = 0 (empty, N=0, S=0),
  1 (doublet, N=1, S=1/2), 2 (doubly occupied, N=2, S=0).
* The two-site block is (k, k+1).  Bonds 0..k are *left* bonds: a sector is the
  (N, 2S) of the block of sites 0..b-1.  Bonds k+2..n are *right* bonds: a
  sector is the (N, 2S) of the block of sites b..n-1.  Bond 0 and bond n each
  hold the single sector (0, 0, dim 1).
* Left site tensor A[j] (j < k): blocks (l, sigma, a), l a sector of left bond
  j, a a sector of left bond j+1, N_a = N_l + N_sigma, triangle(S_l, s_sigma,
  S_a); block shape D_l x D_a.  State |a beta> = sum A[alpha, beta]
  |(l_alpha sigma) S_a> with the l-block to the left of the site in
  creation-operator order and Clebsch-Gordan order (l, sigma).  For every a the
  stacked matrix over (l, sigma) has orthonormal columns.
* Right site tensor B[j] (j >= k+2): blocks (c, sigma, r), c a sector of right
  bond j, r a sector of right bond j+1, N_c = N_sigma + N_r, triangle(s_sigma,
  S_r, S_c); block shape D_c x D_r.  State |c alpha> = sum B[alpha, beta]
  |(sigma r_beta) S_c>, site to the left, CG order (sigma, r).  For every c the
  concatenated matrix over (sigma, r) has orthonormal rows.
* Blocks of a site tensor are ordered by (first sector index, sigma, second
  sector index); each block is row-major.
* Two-site wavefunction psi at (k, k+1), coupled at the middle cut as
  ((l sigma1) S_a, (sigma2 r) S_c) S with CG orders (l, sigma1), (sigma2, r),
  (a, c).  It is stored as super-blocks (a, c): a = (N_a, 2S_a) of the
  enlarged left block, c = (N_c, 2S_c) of the enlarged right block,
  N_a + N_c = N, triangle(S_a, S_c, S); super-blocks sorted by
  (N_a, 2S_a, 2S_c).  A super-block is a dense row-major matrix whose rows are
  the (l, sigma1) sub-blocks sorted by (l index, sigma1) and whose columns are
  the (sigma2, r) sub-blocks sorted by (sigma2, r index); only combinations
  allowed by particle number and the triangle rule, with non-zero dimension,
  appear.  Super-blocks with no rows or no columns are omitted.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

LOCAL = ((0, 0), (1, 1), (2, 0))  # (N, 2s) of sigma = 0, 1, 2


def tri(a2, b2, c2):
    """Triangle rule on doubled spins."""
    return abs(a2 - b2) <= c2 <= a2 + b2 and (a2 + b2 + c2) % 2 == 0


def full_counts(m):
    """Number of multiplets per (N, 2S) in a block of m orbitals, by coupling
    one site at a time (Weyl-Paldus counts)."""
    cur = {(0, 0): 1}
    for _ in range(m):
        nxt = {}
        for (nl, sl), d in cur.items():
            for ns, ss in LOCAL:
                for sa in range(abs(sl - ss), sl + ss + 1, 2):
                    key = (nl + ns, sa)
                    nxt[key] = nxt.get(key, 0) + d
        cur = nxt
    return cur


def _allocate(caps, total_d, nbar, sigma_n, beta):
    keys = [k for k, c in caps.items() if c > 0]
    if not keys:
        return {}
    w = {k: (k[1] + 1) * math.exp(-((k[0] - nbar) ** 2) / (2 * sigma_n ** 2))
         * math.exp(-beta * (k[1] / 2) * (k[1] / 2 + 1)) for k in keys}
    target = min(total_d, sum(caps[k] for k in keys))
    lo, hi = 0.0, 1.0
    while sum(min(caps[k], math.floor(hi * w[k])) for k in keys) < target:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if sum(min(caps[k], math.floor(mid * w[k])) for k in keys) < target:
            lo = mid
        else:
            hi = mid
    dims = {k: min(caps[k], math.floor(lo * w[k])) for k in keys}
    short = target - sum(dims.values())
    order = sorted(keys, key=lambda k: (-(lo * w[k] - math.floor(lo * w[k])), k))
    for k in order:
        if short <= 0:
            break
        if dims[k] < caps[k]:
            dims[k] += 1
            short -= 1
    return {k: v for k, v in dims.items() if v > 0}


@dataclass
class SU2MPS:
    n: int
    n_elec: int
    two_s: int
    k: int
    left_bonds: list                      # b = 0..k : list of (N, 2S, dim)
    right_bonds: dict                     # b = k+2..n : list of (N, 2S, dim)
    A: list = field(default_factory=list)  # j = 0..k-1 : list of (il, sigma, ia, block)
    B: dict = field(default_factory=dict)  # j = k+2..n-1 : list of (ic, sigma, ir, block)

    # ---- flat form handed across the C ABI -------------------------------------------
    def bond_table(self):
        """(sectors [n_bonds_total, 3] int32, counts [n+1] int32) for bonds 0..n,
        with bond k+1 (inside the two-site block) left empty."""
        secs, counts = [], []
        for b in range(self.n + 1):
            if b <= self.k:
                lst = self.left_bonds[b]
            elif b >= self.k + 2:
                lst = self.right_bonds[b]
            else:
                lst = []
            counts.append(len(lst))
            secs.extend(lst)
        return np.asarray(secs, dtype=np.int32).reshape(-1, 3), np.asarray(counts, dtype=np.int32)

    def site_blocks_flat(self):
        """All site tensors concatenated: sites 0..k-1 then k+2..n-1, each in
        canonical block order, each block row-major (float64)."""
        parts = []
        for j in range(self.k):
            parts.extend(blk.ravel() for (_, _, _, blk) in self.A[j])
        for j in range(self.k + 2, self.n):
            parts.extend(blk.ravel() for (_, _, _, blk) in self.B[j])
        return np.concatenate(parts) if parts else np.zeros(0)


def left_site_blocks(lb, ab):
    """Allowed (il, sigma, ia) for a left site between bond sectors lb and ab."""
    out = []
    for il, (nl, sl, dl) in enumerate(lb):
        for s, (ns, ss) in enumerate(LOCAL):
            for ia, (na, sa, da) in enumerate(ab):
                if na == nl + ns and tri(sl, ss, sa) and dl > 0 and da > 0:
                    out.append((il, s, ia))
    return out


def right_site_blocks(cb, rb):
    """Allowed (ic, sigma, ir) for a right site between bond sectors cb and rb."""
    out = []
    for ic, (nc, sc, dc) in enumerate(cb):
        for s, (ns, ss) in enumerate(LOCAL):
            for ir, (nr, sr, dr) in enumerate(rb):
                if nc == ns + nr and tri(ss, sr, sc) and dc > 0 and dr > 0:
                    out.append((ic, s, ir))
    return out


def psi_layout(lb, rb, n_elec, two_s):
    """Super-block layout of the two-site wavefunction (see module docstring).

    Returns a list of super-blocks, each a dict with keys
    'a' (N_a, 2S_a), 'c' (N_c, 2S_c), 'rows' [(il, sigma1, offset, D_l)],
    'cols' [(sigma2, ir, offset, D_r)], 'nrows', 'ncols', 'offset'.
    """
    a_keys = sorted({(nl + ns, sa) for (nl, sl, dl) in lb for (ns, ss) in LOCAL
                     for sa in range(abs(sl - ss), sl + ss + 1, 2) if dl > 0})
    c_keys = sorted({(ns + nr, sc) for (nr, sr, dr) in rb for (ns, ss) in LOCAL
                     for sc in range(abs(ss - sr), ss + sr + 1, 2) if dr > 0})
    blocks, off = [], 0
    for (na, sa) in a_keys:
        for (nc, sc) in c_keys:
            if na + nc != n_elec or not tri(sa, sc, two_s):
                continue
            rows, r0 = [], 0
            for il, (nl, sl, dl) in enumerate(lb):
                for s1, (ns, ss) in enumerate(LOCAL):
                    if nl + ns == na and tri(sl, ss, sa) and dl > 0:
                        rows.append((il, s1, r0, dl))
                        r0 += dl
            cols, c0 = [], 0
            for s2, (ns, ss) in enumerate(LOCAL):
                for ir, (nr, sr, dr) in enumerate(rb):
                    if ns + nr == nc and tri(ss, sr, sc) and dr > 0:
                        cols.append((s2, ir, c0, dr))
                        c0 += dr
            if r0 == 0 or c0 == 0:
                continue
            blocks.append(dict(a=(na, sa), c=(nc, sc), rows=rows, cols=cols,
                               nrows=r0, ncols=c0, offset=off))
            off += r0 * c0
    return blocks


def psi_size(layout):
    return sum(b["nrows"] * b["ncols"] for b in layout)


def random_mps(n, n_elec, two_s, d_max, k=None, seed=0, sigma_n=3.0, beta=0.15):
    """Random mixed-canonical SU(2) MPS for the two-site block (k, k+1).

    Bond dimensions (multiplets) follow a sector model: sector (N, S) of a
    block of b orbitals gets weight (2S+1) exp(-(N - N b/n)^2 / 2 sigma_n^2)
    exp(-beta S(S+1)); d_max multiplets are shared in proportion to the
    weights, capped by the exact number of multiplets the block can hold, by
    the number the other side of the chain can pair with, and by what the
    neighbouring bond can feed through one site (so every tensor can be an
    isometry).
    """
    if k is None:
        k = n // 2 - 1
    assert 0 <= k <= n - 2
    rng = np.random.default_rng(seed)
    counts = [full_counts(m) for m in range(n + 1)]

    def cap_vs_right(b, nl, sl):
        m = n - b
        return sum(counts[m].get((n_elec - nl, sr), 0)
                   for sr in range(abs(sl - two_s), sl + two_s + 1, 2))

    def cap_vs_left(b, nr, sr):
        return sum(counts[b].get((n_elec - nr, sl), 0)
                   for sl in range(abs(sr - two_s), sr + two_s + 1, 2))

    left = [[(0, 0, 1)]]
    for b in range(1, k + 1):
        feed = {}
        for (nl, sl, dl) in left[-1]:
            for ns, ss in LOCAL:
                for sa in range(abs(sl - ss), sl + ss + 1, 2):
                    feed[(nl + ns, sa)] = feed.get((nl + ns, sa), 0) + dl
        caps = {key: min(v, cap_vs_right(b, *key)) for key, v in feed.items()}
        dims = _allocate(caps, d_max, n_elec * b / n, sigma_n, beta)
        left.append([(nk, sk, dims[(nk, sk)]) for (nk, sk) in sorted(dims)])

    right = {n: [(0, 0, 1)]}
    for b in range(n - 1, k + 1, -1):
        feed = {}
        for (nr, sr, dr) in right[b + 1]:
            for ns, ss in LOCAL:
                for sc in range(abs(ss - sr), ss + sr + 1, 2):
                    feed[(ns + nr, sc)] = feed.get((ns + nr, sc), 0) + dr
        caps = {key: min(v, cap_vs_left(b, *key)) for key, v in feed.items()}
        dims = _allocate(caps, d_max, n_elec * (n - b) / n, sigma_n, beta)
        right[b] = [(nk, sk, dims[(nk, sk)]) for (nk, sk) in sorted(dims)]

    mps = SU2MPS(n=n, n_elec=n_elec, two_s=two_s, k=k, left_bonds=left, right_bonds=right)
    for j in range(k):
        lb, ab = left[j], left[j + 1]
        allowed = left_site_blocks(lb, ab)
        blocks = {}
        for ia, (na, sa, da) in enumerate(ab):
            rows = [(il, s) for (il, s, x) in allowed if x == ia]
            nrow = sum(lb[il][2] for il, _ in rows)
            q, _ = np.linalg.qr(rng.normal(size=(nrow, da)))
            r0 = 0
            for il, s in rows:
                dl = lb[il][2]
                blocks[(il, s, ia)] = q[r0:r0 + dl, :].copy()
                r0 += dl
        mps.A.append([(il, s, ia, blocks[(il, s, ia)]) for (il, s, ia) in allowed])
    for j in range(n - 1, k + 1, -1):
        cb, rb = right[j], right[j + 1]
        allowed = right_site_blocks(cb, rb)
        blocks = {}
        for ic, (nc, sc, dc) in enumerate(cb):
            cols = [(s, ir) for (x, s, ir) in allowed if x == ic]
            ncol = sum(rb[ir][2] for _, ir in cols)
            q, _ = np.linalg.qr(rng.normal(size=(ncol, dc)))
            qt = q.T
            c0 = 0
            for s, ir in cols:
                dr = rb[ir][2]
                blocks[(ic, s, ir)] = qt[:, c0:c0 + dr].copy()
                c0 += dr
        mps.B[j] = [(ic, s, ir, blocks[(ic, s, ir)]) for (ic, s, ir) in allowed]
    return mps


def random_psi(mps, seed=1):
    """Random normalised two-site wavefunction in the super-block layout."""
    lay = psi_layout(mps.left_bonds[mps.k], mps.right_bonds[mps.k + 2], mps.n_elec, mps.two_s)
    rng = np.random.default_rng(seed)
    v = rng.normal(size=psi_size(lay))
    return v / np.linalg.norm(v), lay
