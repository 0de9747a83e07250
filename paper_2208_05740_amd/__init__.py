"""MI355X-native GCP-CROWN bound propagation (arXiv 2208.05740).

The compute path is the HIP library libgcp.so (C ABI in include/gcp.h);
``paper_2208_05740_amd.binding`` marshals torch device tensors into it.
Importing the package does not load the library; ``binding.lib()`` does and
raises if it is missing.
"""
__all__ = ["binding", "build"]
