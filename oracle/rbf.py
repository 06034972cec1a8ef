"""RBF kernel K(u, v) = exp(-(u - v)^2 / sigma^2) and its derivatives (oracle).

Paper: Sec. 3 (kernel definition and the derivative operator nabla^a_c K,
the closed forms for the first and second derivative in the first argument).
sigma is the bandwidth itself: the kernel divides by sigma^2.

With z = (u - v) / sigma and g(x) = exp(-x^2/sigma^2),
    d^k/dx^k g(x) = (-1/sigma)^k H_k(z) exp(-z^2)
where H_k is the physicists' Hermite polynomial (H_0 = 1, H_1 = 2z,
H_{k+1} = 2z H_k - 2k H_{k-1}).  Because K(u, v) = g(u - v),
    d^a/du^a d^c/dv^c K = (-1)^c g^{(a+c)}(u - v) = (-1)^a sigma^{-(a+c)} H_{a+c}(z) e^{-z^2}.
For a = 1, 2 and c = 0 this is the paper's pair of closed forms.
"""
import numpy as np


def hermite(k, z):
    """Physicists' Hermite polynomial H_k(z) by the three-term recurrence."""
    z = np.asarray(z, dtype=np.float64)
    h_prev = np.ones_like(z)
    if k == 0:
        return h_prev
    h = 2.0 * z
    for j in range(1, k):
        h_prev, h = h, 2.0 * z * h - 2.0 * j * h_prev
    return h


def kernel(u, v, sigma):
    """K(u, v) = exp(-(u - v)^2 / sigma^2), broadcasting u against v."""
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    return np.exp(-((u - v) ** 2) / sigma ** 2)


def kernel_du(a, u, v, sigma):
    """d^a/du^a K(u, v): derivative in the evaluation (first) argument."""
    return kernel_mixed(a, 0, u, v, sigma)


def kernel_mixed(a, c, u, v, sigma):
    """d^a/du^a d^c/dv^c K(u, v) = (-1)^a sigma^{-(a+c)} H_{a+c}(z) exp(-z^2)."""
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    z = (u - v) / sigma
    return (-1.0) ** a * sigma ** (-(a + c)) * hermite(a + c, z) * np.exp(-z * z)


def kernel_du_dsigma(a, u, v, sigma):
    """d/dsigma of d^a/du^a K(u, v).

    Differentiating (-1/sigma)^a H_a(z) e^{-z^2} with dz/dsigma = -z/sigma and
    H_a' - 2z H_a = -H_{a+1} gives (-1)^{a+1} sigma^{-a-1} e^{-z^2} (a H_a - z H_{a+1}).
    """
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    z = (u - v) / sigma
    return ((-1.0) ** (a + 1) * sigma ** (-a - 1) * np.exp(-z * z)
            * (a * hermite(a, z) - z * hermite(a + 1, z)))
