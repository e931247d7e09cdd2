"""Device buffers for GPU tests through the HIP runtime the library itself links, not torch: a torch
imported after the library would share its runtime by soname and find no device."""
import ctypes

import numpy as np

from paper_2404_11631_amd import sim


class Hip:
    """hipMalloc'd buffers, filled with a byte pattern, copied back on demand and freed by close()."""

    def __init__(self):
        self.ct = ctypes
        sim.load()
        self.L = ctypes.CDLL("libamdhip64.so.7")
        vp = ctypes.c_void_p
        self.L.hipMalloc.argtypes = [ctypes.POINTER(vp), ctypes.c_size_t]
        self.L.hipFree.argtypes = [vp]
        self.L.hipMemcpy.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_int]
        self.L.hipMemset.argtypes = [vp, ctypes.c_int, ctypes.c_size_t]
        self.bufs = []

    def alloc(self, nbytes, fill=0xFF):
        p = self.ct.c_void_p()
        assert self.L.hipMalloc(self.ct.byref(p), nbytes) == 0
        assert self.L.hipMemset(p, fill, nbytes) == 0
        self.bufs.append(p)
        return p.value

    def get(self, ptr, dtype, n):
        a = np.empty(n, dtype=dtype)
        assert self.L.hipDeviceSynchronize() == 0
        assert self.L.hipMemcpy(a.ctypes.data, ptr, a.nbytes, 2) == 0    # device to host
        return a

    def close(self):
        for p in self.bufs:
            self.L.hipFree(p)
