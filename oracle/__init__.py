"""FP64 CPU oracle for the NFFT nonlocal-denoising hot path (arXiv 2407.06834).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link or run
anything under ``oracle/``: only the tests, the smoke check and the CPU-baseline leg of
the benchmark use it.  It shares no code, table or constant generator with the HIP
library; the only common inputs are the seeded images of ``synth``, passed in as arrays.

Modules
  features  per-pixel features and the fixed window grouping (Sec. 5, feature windows)
  kernel    dense / direct-sum extended Gaussian ANOVA kernel, D, eta, L, A (Sec. 2.6)
  nfft      NFFT-based fast Gauss summation, written step by step (Sec. 3), plus NDFT
  solve     dense Cholesky solve and the deflated Jacobi PCG in the paper's U basis and in
            the equivalent projector form (Sec. 4.2, 4.3, 5.3-5.4)
  csum      C/OpenMP direct sums of kernel rows (large N, sampled rows)
  mis       mutual-information ranking of the features into windows (Sec. 5)
  cnn       the warm-start network (not from the paper)

Every function names the passage of the paper it follows.  Functions whose result has no
independent pin are marked "parity unpinned" in their docstring.
"""
