"""MI355X-native separable N-point correlation function estimator
(Philcox & Slepian, arXiv:2106.10278): HIP kernels behind a C ABI."""
