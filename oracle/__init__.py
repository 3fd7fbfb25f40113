"""FP64 CPU oracle for the minor-cycle FISTA path of the two-step reconstruction.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, tables, constants or helpers); the only thing both sides
consume is the seeded input generator in ``synth``.

It is written to be read against the paper (Wang, Prunet, Mignot, Ferrari,
"Multi-Step Reconstruction of Radio-Interferometric Images"):

* ``conv``        -- the PSF convolution operator H and its adjoint
                     (Sect. 3.2, the operator H_L; Sect. 3.3, H_H), with a
                     brute-force spatial sum, a separable direct DFT and an
                     FFT back-end.
* ``filters``     -- the low/high-pass filter responses g_L, g_H (Eqs. 6-10).
* ``objectives``  -- the step-1 and step-2 objectives (Eqs. 4, 5) and their
                     gradients (Eqs. 11, 12).
* ``fista``       -- soft thresholding and FISTA with the (k-1)/(k+2)
                     momentum (Algorithm 1).
* ``lipschitz``   -- the Lipschitz constant theta = 2 lambda_max by power
                     iteration and its closed form for circular convolutions
                     (Sect. 3.4).
* ``helpers``     -- sigma^2 / eta^2 estimators (Sect. 4.3), the lambda
                     schedule (Sect. 5 and App. A.2), the low-resolution
                     image (Sect. 3.2) and PSNR.
* ``twostep``     -- both steps in sequence and their major cycles with
                     image-domain residuals (Sect. 3.2, 3.3).
* ``wavelets``    -- the dictionary W of Daubechies bases db1 .. db8
                     (Sect. 3, App. A.1).
* ``unet``        -- the learned warm start: a small U-Net with bfloat16
                     storage, its forward pass, loss and gradients.
* ``downsample``  -- the down-sampled low-resolution image: decimation D,
                     up-sampling U and the small-grid filter term (Sect. 6.1).

Every floating-point computation runs in float64 unless a caller asks for
float32 (used only to time a float32 CPU variant).
"""
from . import conv, filters, objectives, fista, lipschitz, helpers, twostep  # noqa: F401
