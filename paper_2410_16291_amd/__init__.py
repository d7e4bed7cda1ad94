"""MI355X-native integral image (summed-area table) and sliding-window statistics.

The compute path is the HIP library libsat.so (kernels for gfx950 behind a C ABI declared in
include/sat.h).  This package is its thin Python face: `api` marshals torch tensors into the C
calls, `synth` makes seeded synthetic inputs, `batch`, `autotune` and `serve` add the batched
launch, the tile-shape tuner and the serving loop.  Importing the package loads nothing; the
library is loaded on first use and a missing library is an error, never a fallback.
"""
__all__ = ["api", "synth"]
