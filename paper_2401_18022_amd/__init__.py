"""MI355X-native ISRS GN numerical-integral engine (arXiv:2401.18022 hot path).

Submodules: ``workloads`` (seeded synthetic inputs), ``binding`` (ctypes front-end of
libisrsgn.so), ``autograd`` (torch.autograd.Function for the throughput).
"""
