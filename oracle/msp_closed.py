"""Other FP64 evaluation orders of the same MSP-preconditioned CG, for
iteration bands (oracle).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``: it uses the oracle's
hierarchy and Laplacian and shares nothing with the GPU library.

CG's iteration count in FP64 is not sharp: it moves with how the steps are
rounded.  The oracle applies the MSP by eliminating the sparsifier T~ in the
expanded space (Gaussian elimination, Sec. 3.3) and sums its inner products
left to right.  The same operator also has the closed form obtained by
eliminating T~ aggregate by aggregate, bottom-up, and telescoping the
level weights of P(mu) (Sec. 2.2, Sec. 3.3):

    M = sum_{j=1..l} theta_j P^j D_j^+ (P^j)^T,
    theta_j = s_j^2 mu^(-2(j-1)),  s_j = (1 - (-mu)^j) / (1 + mu),

with P^j the 0/1 aggregation map from level 1 to level j, D_j the block
diagonal of L_B + mu diag(ext) over the aggregates B of level j (ext: the
weight from a node to other aggregates) and D_l = L_l, the top level's
Laplacian (pseudo-inverse).  Its rounding differs from the elimination's:
no term mu^(j-1) is multiplied in and divided out again.

``closed_form(h, mu)`` evaluates that sum with sparse LU per level;
``pcg_exact_sums`` runs the oracle's PCG steps with correctly rounded sums
(math.fsum) for every inner product and mean.  ``band`` is the range of
iteration counts over these evaluation orders and the oracle's rounding
model: a count outside it is not explained by rounding order alone.
"""
import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def closed_form(h, mu):
    """r -> M r - mean(M r) by the closed form above, on an oracle
    Hierarchy ``h`` (levels 0-based here: level k is the paper's k+1)."""
    L = h.nlev
    P = [sp.identity(h.sizes[0], format="csr")]
    for k in range(L - 1):
        agg, _ = h.agg(k)
        nk = len(agg)
        A = sp.csr_matrix((np.ones(nk), (np.arange(nk), agg)), shape=(nk, h.sizes[k + 1]))
        P.append((P[-1] @ A).tocsr())
    terms = []
    for k in range(L):
        ptr, col, w = h.level_csr(k)
        nk = h.sizes[k]
        rows = np.repeat(np.arange(nk), np.diff(ptr))
        if k < L - 1:
            agg, _ = h.agg(k)
            same = agg[rows] == agg[col]
            ext = np.bincount(rows[~same], w[~same], minlength=nk)
            W = sp.csr_matrix((w[same], (rows[same], col[same])), shape=(nk, nk))
            D = sp.diags(np.asarray(W.sum(axis=1)).ravel() + mu * ext) - W
            solve = spla.splu(D.tocsc()).solve
        else:
            W = sp.csr_matrix((w, (rows, col)), shape=(nk, nk)).toarray()
            Pi = np.linalg.pinv(np.diag(W.sum(axis=1)) - W)
            solve = (lambda y, Pi=Pi: Pi @ y)
        j = k + 1
        s = (1.0 - (-mu) ** j) / (1.0 + mu)
        terms.append((s * s * mu ** (-2.0 * (j - 1)), P[k], solve))

    def apply(r):
        z = np.zeros(h.sizes[0])
        for theta, Pk, solve in terms:
            z += theta * (Pk @ solve(Pk.T @ r))
        return z - z.mean()

    return apply


def pcg_exact_sums(g, M, b, tol, maxit, noise=0.0, seed=0):
    """The oracle's PCG steps (x0 = 0, z = M r - mean, stop at ||r|| <=
    tol ||b^||) with every inner product and mean summed by math.fsum.
    noise > 0 applies the oracle's rounding model on top: every L p and
    every M r multiplied entrywise by (1 + noise u), u uniform in [-1, 1)
    (numpy's generator seeded with `seed`).  Returns (iterations, x)."""
    rng = np.random.default_rng(seed)

    def dot(a, c):
        return math.fsum(a * c)

    def mean(a):
        return math.fsum(a) / len(a)

    def perturb(a):
        if noise > 0.0:
            a = a * (1.0 + noise * (2.0 * rng.random(len(a)) - 1.0))
        return a

    bh = b - mean(b)
    nb = math.sqrt(dot(bh, bh))
    x = np.zeros(len(b))
    if nb == 0.0:
        return 0, x
    r = bh.copy()
    z = perturb(M(r))
    z = z - mean(z)
    p = z.copy()
    rho = dot(r, z)
    it = 0
    while it < maxit:
        q = perturb(g.apply(p))
        a = rho / dot(p, q)
        x += a * p
        r -= a * q
        it += 1
        if math.sqrt(dot(r, r)) <= tol * nb:
            break
        z = perturb(M(r))
        z = z - mean(z)
        rho2 = dot(r, z)
        p = z + (rho2 / rho) * p
        rho = rho2
    return it, x - mean(x)


def band(g, b, tol, maxit, h=None, mu=None, precond=None, seeds=8, noise=4e-16):
    """Iteration counts of the same solve under different FP64 rounding.

    precond: an oracle MSP (then h and mu give its closed form too), another
    callable r -> z (e.g. the PEGP of oracle.pegp), or None (plain CG).
    Returns a dict: 'oracle' the plain oracle count, 'runs' a list of
    (label, count) for
      * the oracle (elimination for MSP, sequential sums) and ``seeds`` runs
        of its rounding model (relative noise ``noise`` on L p and M r);
      * the same solve with every sum correctly rounded;
      * for MSP, the closed form under both of the above;
    and 'lo', 'hi' their range."""
    from . import pcg
    runs = []
    variants = [("elim" if precond is not None else "none", precond)]
    if h is not None and mu is not None:
        variants.append(("closed", closed_form(h, mu)))
    for tag, M in variants:
        runs.append((tag, pcg(g, b, tol, maxit, M).iterations))
        runs += [(f"{tag}+noise{s + 1}", pcg(g, b, tol, maxit, M, noise=noise, seed=s + 1).iterations)
                 for s in range(seeds)]
        if M is None:
            Mf = (lambda r: r.copy())
        elif hasattr(M, "apply"):
            Mf = M.apply
        else:
            Mf = M
        runs.append((f"{tag}+exact_sums", pcg_exact_sums(g, Mf, b, tol, maxit)[0]))
    its = [k for _, k in runs]
    return dict(oracle=runs[0][1], runs=runs, lo=min(its), hi=max(its))
