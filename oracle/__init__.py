"""CPU oracle for the FFBS worldline sweep — TEST INFRASTRUCTURE, NOT PRODUCT CODE.

A plain, slow, FP64 NumPy implementation of what one sweep of the determinant-free
auxiliary-field sampler computes (Kong, Feng, Xie, Wu, "FFT-Accelerated Auxiliary Variable
MCMC for Fermionic Lattice Models"). It exists only to check the GPU library: tests/,
the smoke check and the benchmark's CPU-baseline leg may import it; the product path never
does, and the oracle shares no code with the GPU library (only the seeded input recipes in
`synth` serve both).

Readings of the paper taken here (each is also listed with its reason in the design notes):
  * Worldlines live in the site basis. The transfer kernel of eq. Tkk is the same linear
    operator as a real-space convolution with G = F^-1[exp(-dtau eps_k)], followed by the
    diagonal potential weight W_l(r) (Sec. 3.3); in the site basis every path weight is
    positive, and the Gibbs conditionals of Sec. 3.5.4/3.5.5 use site occupations.
  * Trotter placement: under the periodic trace (Sec. 3.1) the symmetric split of eq. trotter
    is cyclically equal to prod_l (e^{-dtau K} W_l); a path weighs
    prod_l W_l(r_l) G(r_{l+1} - r_l).
  * Permutations are the identity (each worldline closes on itself) unless a reconnection
    permutation is passed (FFBS, local updates and the pair swaps of `perm` accept one).
  * Convolutions are direct O(N^2) sums with a dense circulant matrix; no FFT anywhere.

Modules: lattice (kernel tables), hs (potentials and field priors), philox (counter RNG),
ffbs (forward filter / backward sampler), gibbs (field conditionals), sweep (composition),
grad (log Z_path and its adjoint), local (local link updates, Sec. 3.5.1), measure
(equal-time observables, Sec. 4), mala (gradient-informed Gaussian-field proposals), perm
(reconnections at tau = beta and their sign, Sec. 3.5.6).
"""
from . import lattice, hs, philox, ffbs, gibbs, sweep, grad, local, measure, mala, perm  # noqa: F401
