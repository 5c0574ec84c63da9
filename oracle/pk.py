"""Binned power spectrum and its covariance across realizations.
Test infrastructure only.

Sec. 3.2 of the paper estimates the spectrum of a map phi by a DFT, squaring
the modulus and averaging over the modes of a shell (eq. Def spec):
P^(l) = (1/V) (1/N_l) sum_{l' in shell} |phi~(l')|^2, phi~ the Fourier
transform with the cell area as measure, V the survey area.  For counts the
map is the galaxy contrast delta_g = (N/f - N^)/N^ on unmasked cells (zero
where f = 0) with N^ = N_tot / sum f (eq. Estim); no shot noise is
subtracted.  The spectrum covariance is estimated from many realizations and
normalised as C_ab = <P_a P_b> / (<P_a><P_b>) - 1 (the matrix in eq. cuminfo).

With phi~(q) = h^d F(q), F the plain DFT sum_x phi(x) exp(-2 pi i q.x / N), and
V = N^d h^d this is P^_b = (h^d / N^d) mean_{q in b} |F(q)|^2.

Readings taken here:

* Shells are linear in |k| on (0, k_Ny], k_Ny = pi / h (the pixel scale of
  Sec. 3.3): mode q (signed frequencies q~_i = q_i for q_i <= N_i/2, else
  q_i - N_i) is in shell b when b < nb |k| / k_Ny <= b + 1, i.e. |k| / k_Ny =
  2 sqrt(sum_i (q~_i / N_i)^2).  Evaluated exactly in integers: with L the
  least common multiple of the N_i, b + 1 is the smallest s >= 0 with
  s^2 L^2 >= sum_i 4 nb^2 (L / N_i)^2 q~_i^2 (for a cubic grid, s^2 N^2 >=
  4 nb^2 |q~|^2).  The DC mode and corner modes beyond k_Ny are in no shell.
* Rectangular cells (sides h_i): |k|^2 = sum_i (2 pi q~_i / (N_i h_i))^2, shells linear on
  (0, pi / h_ref] with h_ref = max h_i (the largest |k| that every axis resolves).  With
  h_i = h_ref a_i / c_i (a_i / c_i the fraction of smallest denominator c_i <= 64 equal to
  h_i / h_ref within 1e-12; other ratios are not supported) and D = lcm(N_i a_i), the
  integers are t = sum_i 4 nb^2 (c_i D / (N_i a_i))^2 q~_i^2 against (s D)^2; equal sides
  give a_i = c_i = 1, D = L and the rule above.  The paper bins in ln l:
  any ascending shell edges e_b in |k| may be given instead; then, with t the
  integer above (t = nb^2 L^2 (|k| / k_Ny)^2), a mode is in shell b when
  TH_b < t <= TH_{b+1}, TH_b = nb^2 L^2 (e_b h / pi)^2 in FP64, snapped to an
  integer within 1e-9 relative and rounded down otherwise (edges linear on
  (0, k_Ny] give the integer rule back).
* N_b counts every full-grid mode (q and -q separately).
* Covariance across R realizations: the unbiased Cov_ab with 1/(R - 1), and
  the paper's normalised C_ab with 1/R sample means.

Parity: pinned by Parseval's identity, the single-plane-wave closed form, the
white-noise level, a brute-force shell enumeration in Python integers, the
closed-form expected survey power of a Gaussian field, and numpy.cov; the cumulative
information by its diagonal closed form (half the number of modes for Gaussian shells), a
2x2 closed form and its scaling.  See ``tests/test_oracle_pk.py``.
"""

import math

import numpy as np


def signed_freq(n):
    """q~ = q for q <= n/2, q - n otherwise."""
    q = np.arange(n)
    return np.where(q <= n // 2, q, q - n)


def cell_ratios(h, d):
    """(h_ref, a, c): h_ref = max h_i and h_i / h_ref = a_i / c_i, the fraction of smallest
    denominator c_i <= 64 within 1e-12 relative (ValueError when there is none)."""
    hs = tuple(float(x) for x in h) if np.ndim(h) else (float(h),) * d
    href = max(hs)
    a, c = [], []
    for x in hs:
        rho = x / href
        for den in range(1, 65):
            num = round(rho * den)
            if num >= 1 and abs(num - rho * den) <= 1e-12 * rho * den:
                a.append(num)
                c.append(den)
                break
        else:
            raise ValueError("cell sides %r: ratio %r is not a fraction with denominator <= 64" % (hs, rho))
    return href, a, c


def grid_weights(n, h):
    """(D, w, h_ref): |k| / (pi / h_ref) = 2 sqrt(sum_i (w_i q~_i)^2) / D with integer weights
    w_i = c_i D / (N_i a_i) and D = lcm(N_i a_i) (square cells: D = lcm(N_i), w_i = D / N_i)."""
    n = tuple(int(x) for x in n)
    href, a, c = cell_ratios(h, len(n))
    D = 1
    for x, ai in zip(n, a):
        D = D * (x * ai) // math.gcd(D, x * ai)
    return D, [ci * (D // (x * ai)) for x, ai, ci in zip(n, a, c)], href


def shell_thresholds(n, h, nbins, edges):
    """Integer thresholds of user shell edges (|k| values e_0 < ... < e_nb): a mode with the
    integer t below is in shell b when TH_b < t <= TH_{b+1} (t = nb^2 D^2 (|k| / k_Ny)^2,
    k_Ny = pi / h_ref).  TH_b is v = nb^2 D^2 (e_b h_ref / pi)^2 evaluated in FP64 in this
    order, rounded to the nearest integer when it lies within 1e-9 v of one (an edge placed on
    a mode by an FP64 formula, e.g. linear edges, keeps the mode in the lower shell as the
    integer rule does) and rounded down otherwise."""
    n = tuple(int(x) for x in n)
    L, _, href = grid_weights(n, h)
    scale = float(int(nbins) ** 2 * L * L)
    out = []
    for e in edges:
        x = float(e) * float(href) / math.pi
        v = scale * (x * x)
        r = math.floor(v + 0.5)
        out.append(int(r) if abs(v - r) <= 1e-9 * v else int(math.floor(v)))
    return np.array(out, dtype=np.int64)


def shell_index(n, nbins, edges=None, h=1.0):
    """Shell of every mode of a grid of shape n with cell sides h (a number or one per axis),
    -1 where the mode is in no shell.

    Square cells: |k| / k_Ny = 2 sqrt(sum_i (q~_i / N_i)^2); with L = lcm(N_i) the mode is in
    shell b = s - 1 for the smallest integer s >= 0 with (s L)^2 >= t,
    t = sum_i 4 nb^2 (L / N_i)^2 q~_i^2, decided in integers (a cubic grid has L = N and
    t = 4 nb^2 |q~|^2); rectangular cells use the weights of ``grid_weights`` and D for L.
    With edges (|k| values, nb + 1 ascending) the shells are those of ``shell_thresholds``."""
    n = tuple(int(x) for x in n)
    L, w, _ = grid_weights(n, h)
    grids = np.meshgrid(*[signed_freq(x).astype(np.int64) for x in n], indexing="ij")
    nb2 = 4 * int(nbins) ** 2
    t = sum(nb2 * wi * wi * g * g for wi, g in zip(w, grids))
    if edges is not None:
        th = shell_thresholds(n, h, nbins, edges)
        b = np.searchsorted(th, t, side="left") - 1  # number of thresholds below t, minus one
        return np.where((b >= 0) & (b < nbins), b, -1)
    # r = smallest integer with r*r >= t (exact integer ceil-sqrt)
    r = np.floor(np.sqrt(t.astype(np.float64))).astype(np.int64)
    r = np.where(r * r < t, r + 1, r)
    r = np.where((r - 1) * (r - 1) >= t, r - 1, r)
    r = np.where(r * r < t, r + 1, r)
    s = -(-r // L)  # ceil(r / L): smallest s with s*L >= r
    b = s - 1
    return np.where((b >= 0) & (b < nbins), b, -1)


def shell_stats(n, h, nbins, edges=None):
    """(N_b, mean |k| per shell) for a grid of shape n with cell sides h."""
    n = tuple(int(x) for x in n)
    b = shell_index(n, nbins, edges, h)
    hs = tuple(float(x) for x in h) if np.ndim(h) else (float(h),) * len(n)
    href = max(hs)
    # |k| h_ref = 2 pi sqrt(sum_i ((q~_i / N_i) / (h_i / h_ref))^2)
    grids = np.meshgrid(*[(signed_freq(x).astype(np.float64) / x) / (hi / href) for x, hi in zip(n, hs)],
                        indexing="ij")
    kmag = 2.0 * np.pi * np.sqrt(sum(g * g for g in grids)) / href
    sel = b >= 0
    nmodes = np.bincount(b[sel], minlength=nbins).astype(np.int64)
    ksum = np.bincount(b[sel], weights=kmag[sel], minlength=nbins)
    with np.errstate(invalid="ignore", divide="ignore"):
        kmean = ksum / nmodes
    return nmodes, kmean


def contrast_from_counts(counts, ntot=None, mask=None):
    """delta_g = (N/f - N^)/N^ on f != 0, zero elsewhere; N^ = N_tot / sum f (eq. Estim)."""
    counts = np.asarray(counts, dtype=np.float64)
    f = np.ones_like(counts) if mask is None else np.asarray(mask, dtype=np.float64)
    tot = counts.sum() if ntot is None else float(ntot)
    nhat = tot / f.sum()
    out = np.zeros_like(counts)
    on = f != 0
    out[on] = (counts[on] / f[on] - nhat) / nhat
    return out


def power_spectrum(phi, h, nbins, edges=None):
    """P^_b = (prod_i h_i / N^d) mean_{q in b} |F(q)|^2 for one map phi (eq. Def spec; h a
    number or one cell side per axis)."""
    phi = np.asarray(phi, dtype=np.float64)
    n = phi.shape
    F = np.fft.fftn(phi)
    p2 = (F.real ** 2 + F.imag ** 2)
    b = shell_index(n, nbins, edges, h)
    sel = b >= 0
    nmodes = np.bincount(b[sel], minlength=nbins)
    sums = np.bincount(b[sel], weights=p2[sel], minlength=nbins)
    with np.errstate(invalid="ignore", divide="ignore"):
        mean = sums / nmodes
    cell = float(np.prod([float(x) for x in h])) if np.ndim(h) else float(h) ** phi.ndim
    return (cell / float(np.prod(n))) * mean


def estimate_pk(maps, h, nbins, kind="field", ntot=None, mask=None, edges=None):
    """Spectra of a stack of maps (count, *N).  kind: 'field' or 'counts'; edges: optional shell
    edges in |k| (nb + 1 ascending), e.g. logarithmic as in the paper."""
    maps = np.asarray(maps)
    out = np.empty((maps.shape[0], nbins), dtype=np.float64)
    for k in range(maps.shape[0]):
        if kind == "counts":
            phi = contrast_from_counts(maps[k], None if ntot is None else ntot[k], mask)
        else:
            phi = maps[k]
        out[k] = power_spectrum(phi, h, nbins, edges)
    return out


def covariance(pk):
    """(Cov with 1/(R-1), paper-normalised C with 1/R means) of spectra pk (R, nb)."""
    pk = np.asarray(pk, dtype=np.float64)
    R = pk.shape[0]
    mean = pk.sum(axis=0) / R
    d = pk - mean
    cov = (d.T @ d) / (R - 1)
    second = (pk.T @ pk) / R
    cpaper = second / np.outer(mean, mean) - 1.0
    return cov, cpaper


def cumulative_information(C):
    """I(<= l_k) = sum of the elements of the inverse of the leading k x k block of the
    normalised covariance C, for k = 1 .. nb (eq. cuminfo)."""
    C = np.asarray(C, dtype=np.float64)
    return np.array([np.linalg.inv(C[:k, :k]).sum() for k in range(1, C.shape[0] + 1)])
