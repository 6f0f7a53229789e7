"""CPU oracle for Variable Basis Mapping (VBM) and its image-space fine-tuning loop.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 restatement of what the
method computes, written from the paper's definitions.  Only the tests, the smoke check
and the benchmark's CPU-baseline leg may import it; the product library never does, and
the two share no code (only the seeded input generators in ``vbm_inputs``).

Modules and the passages they follow:
  wavelets   filter banks: Haar and the CDF 9/7 ("bior4.4") pair derived from the
             Daubechies Bezout polynomial (Sec. 4.2 uses bior4.4; Sec. 3 3D wavelet transform)
  tf         piecewise-linear transfer function RF = TF(F)            (Sec. 3, Transfer Function)
  dwt        periodised separable J-level 3D DWT and its inverse       (Sec. 3; Sec. 4.3, eq. mul_wavelet_coff)
  bank       canonical wavelets, dominant-lobe moments, ridge weight   (Sec. 4.2: eq. canonical_wavelet,
             eq. roi, eq. moment, eq. canonical_gaussian, eq. ridge_regression)
  select     joint-norm global top-K                                   (Supp. A, joint magnitude)
  adaptive   adaptive per-subband selection: budgets, MAD threshold,   (Supp. A: budget allocation,
             capped top-K per subband                                   joint sparsification, MAD, top-K)
  construct  per-coefficient Gaussians                                 (Sec. 4.3: eq. per_location_weight,
             eq. wavelet_gaussian_kernel, eq. translation_operator)
  binning    FP32 projection decisions (depth keys, tile rects) and the sorted pair lists
  render     FP64 EWA projection, front-to-back compositing and its exact gradient
             (Sec. 3, 3D Gaussian Splatting; Sec. 4.4 fine-tuning)
  loss       L1 and SSIM image losses (Sec. 4.4, loss "as in 3DGS")
  adam       Adam update on raw parameters (Sec. 5, Implementation Details)
  dvr        ray-marching direct volume renderer for the supervision images (Sec. 4.4)

Parity unpinned (no printed value or closed form exists): the bior4.4 bank values (u, Sigma, w),
the initial opacity/colour scale (depends on the reading of s_j), absolute PSNRs.
"""
