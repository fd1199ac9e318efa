"""FP64 CPU oracle for the memory-efficient INR gradient step.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product path
(the HIP library and its Python binding) never imports, links or calls it,
and this package imports nothing from the product.

It is a plain, slow, literal restatement of what the paper defines:

  * E, the evaluation operator that samples the INR on the FOV-masked grid
    (Sec. III, the decomposition of the projection into P times E);
  * P, a discrete ray-driven (Joseph) projector, built here as an explicit
    sparse matrix so that its transpose is exact by construction
    (Sec. III, P in R^{m x n});
  * the LS residual r = z - y and loss (Sec. II) and the FLS variant
    r = F(z - y) (Sec. II, Sec. III);
  * v = P^T r (Sec. III, chain rule);
  * the subsampled estimator of Eq. (2) and its virtual-loss form, Eq. (3);
  * Algorithm 1 followed by an Adam update (Sec. IV).

Every function is written in float64 with no blocking or fusion beyond what
its definition states.  Functions whose parity is not pinned by an
independent check say "parity unpinned" in their docstring.
"""
