"""MI355X-native bound evaluation for the reduced-space branch and bound of
K-center clustering (Ren et al., arXiv 2301.00061).

The compute path is libkc.so (HIP for gfx950, C ABI in include/kc.h); the
submodule ``api`` only marshals torch tensors into its calls. Importing the
package does not touch the GPU; the first call loads the library and fails
loudly if it has not been built.
"""
from . import _lib  # noqa: F401

__all__ = ["api", "_lib"]
