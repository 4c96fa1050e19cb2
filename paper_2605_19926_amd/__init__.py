"""MI355X-native batched first-person grid-world environments with a raycast
renderer (the method of JAXenstein, Tao & Konidaris), as HIP kernels for gfx950
behind the C-ABI of include/jx.h.

    from paper_2605_19926_amd import jx      # ctypes binding of libjx.so
    python -m paper_2605_19926_amd.build     # builds libjx.so in-tree
"""
__all__ = ["jx", "build"]
