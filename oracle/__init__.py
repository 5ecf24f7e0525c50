"""Plain FP64 CPU oracle for the directional SLSHT -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the package smoke check and the benchmark's CPU-baseline
leg may import or run anything in this package.  The GPU library never calls
it, and it shares no code with the GPU library (no kernels, headers, helpers,
tables or constant generators); the only thing both sides consume is the
seeded input generator in ``paper_1207_5558_amd.inputs``, which holds no
transform arithmetic.

What it computes (Khalid et al., "Fast directional spatially localized
spherical harmonic transform", IEEE TSP 2013):

  * ``sph``     -- spherical harmonics Y_l^m with the Condon-Shortley phase
                   (Section II-A, eq. Eq:Sph_harmonics);
  * ``wigner``  -- Wigner-d functions: the exact value of d^p(pi/2) (Delta)
                   from Wigner's explicit formula in integer arithmetic, and
                   d^p(beta) from the Delta-Fourier identity of the
                   factoring-of-rotations step (Section IV-B,
                   eq. Eq:WignerD_expansion_new); Wigner-D (eq. Eq:Dlm);
  * ``grid``    -- the equiangular SO(3) grid E_L (Section II-D) and the
                   exact beta quadrature weights q(beta) of the discrete
                   inverse (Section IV-A, eq. Eq:sig_reconstruction_discrete);
  * ``slsht``   -- the distribution g(rho; l, m) by direct quadrature of its
                   defining integral (Definition 1, eq. Eq:stft_spatial):
                   rotate the window by Wigner-D sums (eq.
                   eqn:rotation_non_symm), multiply by f on a Gauss-Legendre x
                   uniform-phi grid that integrates the band-limited product
                   exactly, and project onto conj(Y_l^m); the modulated-signal
                   coefficients A^p_q(l,m) = <f Y_p^q, Y_l^m> by the same
                   quadrature; the per-(l, rho) energy sum_m |g|^2; and the
                   inverse through the spectral marginal (Section III-C,
                   eqs. Eq:inversion_1, Eq:inversion_2, with the discrete sum
                   of eq. Eq:sig_reconstruction_discrete).

Readings of the paper used throughout: band-limits are exclusive (f_l^m = 0 for
l >= L_f, h_s^r = 0 for s >= L_h), and the beta axis of the SO(3) grid is
2*pi*b/n_phi for b = 0..(n_phi-1)/2, as in the definition of E_L.
"""
