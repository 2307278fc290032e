"""CPU oracle for the open-rectangular-pipe Poisson solve (Ryne, arXiv:1111.4971).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package: only the tests, the smoke check and the CPU-baseline leg of the
benchmark do.  It shares no code with the HIP implementation.

Everything here is plain FP64 numpy/scipy, written from the paper:

* ``green``     -- the pipe Green function R (Eq. 9), its z-integrated form
                   R_int (Eq. 14-16), the four-term G (Eq. 8) and the sine
                   series G (Eq. 7).
* ``direct``    -- O1: the discretised Green integral summed directly
                   (the Eq. 4 pattern with the four-term G of Eq. 8).
* ``fourterm``  -- O2: the paper's algorithm, Eq. 10, literally: one forward
                   3-D DFT of the padded charge, four mixed-direction Green
                   transforms, four products, four mixed-direction final
                   transforms (Appendix A.4-A.9 conventions).
* ``modespace`` -- O3: an independent solve in the sine eigenbasis of the pipe
                   (Eq. 7), valid when the mesh spans the full aperture.
* ``conv1d``    -- the 1-D zero-padded FFT convolution and correlation of the
                   Appendix (A.1-A.9).
* ``igf_quad``  -- high-precision quadrature of the defining integral Eq. 14.
* ``freespace`` -- the isolated Green function (Eq. 3) and Hockney's one-term
                   FFT convolution (Eq. 5), used for the free-space limit.
* ``gradient``  -- the gradient of the differentiable-optics loss.

Readings of the paper that these functions adopt (each is also listed in the
design notes):

* Normalisation: R carries the prefactor 1/(2 pi a b) printed in Eq. 9, and the
  four-term G of Eq. 8 uses unit coefficients.  (Eq. 7 as printed is exactly
  one quarter of that; see ``green.G_sine_series``.)
* Node positions: 0-based node i sits at X_i = (i+1) h_x, node j at
  Y_j = (j+1) h_y (the paper's 1-based x_i = i h), and z is translation
  invariant, Z_k = k h_z.
* Mode truncation: m = 1..M_x, n = 1..M_y; the truncation is part of the
  definition of the result.
* IGF: Eq. 13-15 in z only, nodal values interpolated by hats with zero
  extension beyond the grid; delta_{w,0} is the Kronecker delta on grid
  distances.
"""
