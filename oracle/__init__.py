"""FP64 CPU oracle for the Dual Forward-Backward ADMM imaging path.

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, obviously correct
NumPy implementation of what the GPU library computes, written from the paper
(Pratley et al., "Distributed and parallel sparse convex optimization for radio
interferometry with PURIFY"). It shares no code with the GPU library and never
imports it. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product path must not.

Modules
  kaiser_bessel  pre-sampled Kaiser-Bessel gridding kernel and its correction
  measurement    Phi = W G F Z S and its adjoint (Section "Radio Interferometric
                 Measurement Equation", eq. matrix_equation), power method
  wavelets       Daubechies filters, periodic 2-D DWT, the SARA dictionary
  prox           soft thresholding, positivity and l2-ball projections
                 (Section "Proximal Operators")
  admm           Dual Forward-Backward ADMM (Algorithm 1), with the local l2 balls
                 (Section "Local Fidelity Constraint ADMM") and a weighted l1
  fista          FISTA for the MAP problem (Algorithm "FISTA")
  primal_dual    Primal-Dual splitting (Algorithm "Primal-Dual Algorithm")
  reweight       the reweighted analysis l1 loop (Section "Sparse Regularization")
  nudft          the direct non-uniform DFT the NUFFT approximates

Parity status of each function is stated in its module header.
"""
