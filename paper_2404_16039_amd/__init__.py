"""pagefem: MI355X-native page-wise small dense linear algebra and P1 finite element
assembly (arXiv 2404.16039), as hand-written HIP kernels behind a C ABI."""
