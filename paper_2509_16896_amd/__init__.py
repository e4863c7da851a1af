"""MI355X (gfx950) implementation of the improved Yau-Yau filter's time step (arXiv 2509.16896).

The filter step runs in libyy.so (HIP kernels behind the C ABI of include/yy.h);
``yy`` is its Python binding, ``filter`` the time loop built on it and
``workloads`` the seeded synthetic inputs.
"""
