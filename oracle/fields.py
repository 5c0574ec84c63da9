"""Gaussian field realizations by circulant embedding.  Test infrastructure only.

Sec. 2 of the paper: draw independent zero-mean Gaussian Fourier modes on the
doubled periodic grid with variance proportional to the ad-hoc spectrum
(eq. Papos2, with the discrete spectrum of eq. Specd), take the inverse DFT,
and keep the survey cells; the restricted field then has exactly the target
covariance xi(x - y) on the grid (eq. thatiswhatwewant and its discrete
counterpart after eq. Specd).

Readings taken here (the paper states only the mode variance):

* Modes are complex, eps = a + i b with a, b independent N(0, 1), one per
  embedding cell, and X(q) = sqrt(M^d lambda(q)) eps(q).  With the normalised
  inverse DFT Z(m) = M^-d sum_q X(q) exp(+2 pi i q.m / M) this gives
  <Z(m) Z*(m')> = 2 c(m - m') and <Z Z> = 0, so Re Z and Im Z are two
  independent fields, each with covariance c.  Realization 2j is Re Z of pair
  j, realization 2j + 1 is Im Z.
* The kept sub-box is m_i in [0, N_i) (the paper allows any sub-box of side L).
* Noise words: Philox4x32-10 with key = seed split in two words and counter
  (p, j, request_id, 0), p = floor(l / 2) where l is the row-major (last axis
  fastest) index of the embedding cell.  Words (x0, x1) give cell 2p's uniforms
  (u1, u2), words (x2, x3) give cell 2p+1's; u = (x + 1/2) 2**-32 and the
  normals come from Box-Muller.

Parity: the linear map noise -> field is pinned by brute force on tiny grids
(A A^T equals the target matrix) and the noise -> field composition by the
empirical covariance over many draws; see ``tests/test_oracle_fields.py``.
"""

import numpy as np

from . import philox


def pair_noise(M, seed, request_id, pair):
    """Complex standard normals eps(q) on the embedding grid of shape M for one pair."""
    M = tuple(int(x) for x in M)
    total = int(np.prod(M))
    if total % 2:
        raise ValueError("embedding must have an even number of cells")
    p = np.arange(total // 2, dtype=np.uint64)
    x0, x1, x2, x3 = philox.philox4x32_10(p, np.uint64(pair), np.uint64(request_id), np.uint64(0),
                                          philox.key_from_seed(seed))
    a_even, b_even = philox.box_muller(philox.u32_to_unit(x0), philox.u32_to_unit(x1))
    a_odd, b_odd = philox.box_muller(philox.u32_to_unit(x2), philox.u32_to_unit(x3))
    eps = np.empty(total, dtype=np.complex128)
    eps[0::2] = a_even + 1j * b_even
    eps[1::2] = a_odd + 1j * b_odd
    return eps.reshape(M)


def field_pair_from_noise(plan, eps):
    """Complex field Z restricted to the survey: Re and Im are two realizations."""
    lam = plan["lam"]
    M = lam.shape
    X = np.sqrt(float(np.prod(M)) * lam) * eps
    Z = np.fft.ifftn(X)
    crop = tuple(slice(0, int(nn)) for nn in plan["n"])
    return Z[crop]


def generate_fields(plan, seed, request_id, first_realization, count):
    """Realizations first_realization .. first_realization + count - 1, shape (count, *N)."""
    if first_realization % 2:
        raise ValueError("first_realization must be even")
    out = np.empty((count,) + tuple(plan["n"]), dtype=np.float64)
    for k in range(0, count, 2):
        pair = (first_realization + k) // 2
        Z = field_pair_from_noise(plan, pair_noise(plan["M"], seed, request_id, pair))
        out[k] = Z.real
        if k + 1 < count:
            out[k + 1] = Z.imag
    return out

