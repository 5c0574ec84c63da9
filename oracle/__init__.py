"""Plain FP64 CPU oracle for the circulant-embedding field generator.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
reference that the GPU path is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with ``paper_1406_6072_amd`` (the HIP path) and
never imports it.

Every function follows the definition in Carron, Wolk & Szapudi (2014),
"On fast generation of cosmological random fields" (arXiv:1406.6072):

* ``embedding``  -- Sec. 2: lag table on the doubled grid, the discrete
  ad-hoc spectrum (eq. Specd) and its non-negativity condition (eq. condition).
* ``filtered``   -- Sec. 3.1 and App. A: the square top-hat cell average of a
  two-point function (eqs. exactformula, xibar, CoolEq) and the lognormal
  target ln(1 + omega) (eq. Lncov), applied to the lag table by ``embedding``.
* ``fields``     -- Sec. 2: independent Gaussian modes with variance set by the
  ad-hoc spectrum (eq. Papos2), inverse DFT, restriction to the survey grid.
* ``lognormal_poisson`` -- Sec. 3.1: lognormal density (eq. Lncov, step i) and
  Poisson sampling of counts (eq. sampling).
* ``pk``         -- Sec. 3.2: power-spectrum estimator (eq. Def spec) on the
  galaxy contrast with the estimated intensity (eq. Estim); spectrum
  covariance, the normalised matrix of eq. cuminfo and the cumulative information.
* ``kspace``     -- Sec. 3.3: the k-space sampling comparator, a periodic box with the
  modes of the continuous spectrum (eq. Periodicboxmodes), DC zeroed.
* ``cic``        -- Sec. 3.4: counts-in-cells histogram, its Poisson-lognormal
  prediction, and the A* map (eq. As).
* ``philox``     -- the counter-based generator that supplies the noise
  (Salmon et al. 2011, Philox4x32-10) and the uniform / Box-Muller maps.

Parity status of each function is listed in its module header.
"""

from . import philox, embedding, filtered, fields, lognormal_poisson, pk, cic, kspace  # noqa: F401
