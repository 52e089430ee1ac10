"""MI355X-native TUfRG flow right-hand side (arXiv:1604.06296), Python binding.

Every step of the computation runs in the native library
(`_lib/libtufrg.so`, HIP kernels for gfx950) behind the C ABI declared in
include/tufrg.h; this module only marshals arguments.  PyTorch provides
device memory and the stream.  Importing works without a GPU; creating a
Context needs the built library and a GPU, and fails loudly otherwise.
"""
from .binding import (MLP, Context, FlowOptions, FlowResult, TufrgError, library_path,  # noqa: F401
                      load_library, mu_from_filling, CHANNELS, IRREPS)

__all__ = ["Context", "MLP", "FlowOptions", "FlowResult", "TufrgError", "load_library",
           "library_path", "mu_from_filling", "CHANNELS", "IRREPS"]
