"""High-precision (mpmath, 50 digits) restatement of the Lemma 1 solve and of the loss on
y_hat, for pinning the FP64 oracle's gradients where FP64 itself is the question.

Paper: Sec. 3 (RBF kernel and its derivatives), App. A.2 (Nystrom feature map from the
eigendecomposition of the landmark Gram), Sec. 3.1 (Lemma 1 system, y_hat = omega^T phi + b).
Written directly from those definitions with mpmath matrices: K_mm = U Lambda U^T,
W = U_r Lambda_r^{-1/2}, g_i = W^T (k^(p)(t_i) - sum_k f_k k^(p-k)(t_i)), the symmetric
(r+1+p) KKT system, LU solve.  Shares no code with the oracle or the GPU path; tiny
instances only (n ~ 60, m ~ 10: about a second per solve).
"""
from mpmath import mp


def _kd(d, u, v, sig):
    """d-th derivative in u of exp(-(u - v)^2 / sig^2): (-1/sig)^d H_d(z) e^{-z^2}."""
    z = (u - v) / sig
    hs = [mp.mpf(1), 2 * z]
    for j in range(1, d):
        hs.append(2 * z * hs[j] - 2 * j * hs[j - 1])
    return (-1 / sig) ** d * hs[d] * mp.exp(-z * z)


def loss(q, gamma=None, sigma=None, dps=50):
    """Mean squared error of y_hat(t_obs) against y_obs for instance q (a workloads dict with
    observations), with gamma / sigma optionally replaced; returns an mpmath number."""
    with mp.workdps(dps):
        p, n, m = int(q["p"]), int(q["n"]), int(q["m"])
        gam = mp.mpf(q["gamma"] if gamma is None else gamma)
        sig = mp.mpf(q["sigma"] if sigma is None else sigma)
        t = [mp.mpf(float(x)) for x in q["t"]]
        lidx = [(2 * s * (n - 1) + (m - 1)) // (2 * (m - 1)) for s in range(m)]
        tl = [t[i] for i in lidx]
        kmm = mp.matrix(m, m)
        for a in range(m):
            for b in range(m):
                kmm[a, b] = _kd(0, tl[a], tl[b], sig)
        ev, vec = mp.eigsy(kmm)
        order = sorted(range(m), key=lambda k: -ev[k])
        lam = [ev[k] for k in order]
        r = sum(1 for x in lam if x > q["tau"] * lam[0])
        w = mp.matrix(m, r)
        for j in range(r):
            for s in range(m):
                w[s, j] = vec[s, order[j]] / mp.sqrt(lam[j])

        def phi(d, u):
            kv = mp.matrix(1, m)
            for s in range(m):
                kv[0, s] = _kd(d, u, tl[s], sig)
            return kv * w

        conds = list(zip(q["cond_d"], q["cond_i"]))
        skip = {int(i) for _, i in conds}
        rows = [i for i in range(n) if i not in skip]
        f = [[mp.mpf(float(x)) for x in row] for row in q["f"].reshape(p, n)]
        g = mp.matrix(len(rows), r)
        c = mp.matrix(len(rows), 1)
        rv = mp.matrix(len(rows), 1)
        for a, i in enumerate(rows):
            row = phi(p, t[i])
            for k in range(1, p + 1):
                row = row - f[k - 1][i] * phi(p - k, t[i])
            for j in range(r):
                g[a, j] = row[0, j]
            c[a] = -f[p - 1][i]
            rv[a] = mp.mpf(float(q["r"][i]))
        nsys = r + 1 + p
        A = mp.matrix(nsys, nsys)
        rhs = mp.matrix(nsys, 1)
        gtg, gtc, gtr = g.T * g, g.T * c, g.T * rv
        for a in range(r):
            for b in range(r):
                A[a, b] = (1 if a == b else 0) + gam * gtg[a, b]
            A[a, r] = A[r, a] = gam * gtc[a]
            rhs[a] = gam * gtr[a]
        A[r, r] = gam * (c.T * c)[0]
        rhs[r] = gam * (c.T * rv)[0]
        for j, (d, i) in enumerate(conds):
            h = phi(int(d), t[int(i)])
            for a in range(r):
                A[a, r + 1 + j] = A[r + 1 + j, a] = h[0, a]
            A[r, r + 1 + j] = A[r + 1 + j, r] = 1 if int(d) == 0 else 0
            rhs[r + 1 + j] = mp.mpf(float(q["v"][j]))
        x = mp.lu_solve(A, rhs)
        alpha = w * mp.matrix([x[j] for j in range(r)])
        b = x[r]
        tot = mp.mpf(0)
        for sj, yj in zip(q["t_obs"], q["y_obs"]):
            s = mp.mpf(float(sj))
            y = b + mp.fsum(_kd(0, s, tl[k], sig) * alpha[k] for k in range(m))
            tot += (y - mp.mpf(float(yj))) ** 2
        return tot / len(q["t_obs"])


def dloss(q, which, rel_step=1e-20, dps=50):
    """Central difference of `loss` in gamma or sigma with a relative step of 1e-20 at 50
    digits: truncation ~1e-40 and cancellation ~1e-30 relative, far below FP64."""
    with mp.workdps(dps):
        x0 = mp.mpf(q[which])
        h = x0 * mp.mpf(rel_step)
        lp = loss(q, **{which: x0 + h}, dps=dps)
        lm = loss(q, **{which: x0 - h}, dps=dps)
        return float((lp - lm) / (2 * h))
