"""CPU oracle for the blockwise 16-point multiplierless approximate DCT.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute this package: only the test-suite, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code, tables or helpers
with the HIP library; both sides only share the seeded input generators of
``synth``.

Everything here is the plain, slow definition of what the method computes,
written from the paper (Silveira et al., "Multiplierless 16-point DCT
approximation for low-complexity image and video coding"), in exact int64
arithmetic for the integer transforms and float64 for real-valued quantities.
Where the library makes a float decision in fp32 (quantisation levels), the
oracle takes the same decision in fp32 as well; a float64 counterpart is kept
beside it.

``adct_oracle``  the transform, its factorisation, the 2D blockwise codec
                 steps, quantisation, reconstruction, SSE/PSNR.
``metrics``      the exact DCT-II and the similarity / coding measures of
                 Section 2.3 (Table 2).
``image_experiment``  zig-zag retention of the first r coefficients and the
                 SSIM index (Section 3.1 as the paper runs it).
``t8``           the 8-point approximation T8 that T is built from, and its
                 8x8 blockwise codec (Section 3.2's second scenario).
``mixed``        mixed 8/16-point coding: per 16x16 region, one 16x16 block
                 or four 8x8 blocks by the lower Lagrangian cost (Section
                 3.2's second scenario).
``comparison``   the WHT and exact-DCT codecs (Tables 1 and 2's comparison
                 transforms through Section 3.1's experiment).
``c/``           the same plain dense definition of the 2D forward and
                 zonal inverse in C (OpenMP over tiles), used as the timed
                 CPU baseline.
"""
