"""MI355X-native multi-scale MPV (Multi-Path-Viterbi) stereo matcher.

The matcher runs in hand-written HIP kernels for gfx950 behind the C ABI of
include/mpv.h (libmpv.so, built in-tree by ``paper_2001_09678_amd.build``). Importing the
package does not load the library; the first call does, and fails loudly if it is
missing. ``scene`` holds the seeded synthetic stereo scenes used as inputs.
"""

__all__ = ["mpv", "scene", "build"]
