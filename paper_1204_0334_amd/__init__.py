"""MI355X-native batched sum-product decoder for quasi-cyclic LDPC block codes
and LDPC convolutional codes (Zhao & Lau, arXiv:1204.0334).

    from paper_1204_0334_amd import ldpc     # the C-ABI binding (needs the built library)
    from paper_1204_0334_amd import build    # compiles csrc/ for gfx950

The decoder itself is the HIP library built from csrc/; `ldpc` only marshals
arguments to it.
"""
__all__ = ["ldpc", "build"]
