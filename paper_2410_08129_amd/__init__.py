"""MI355X-native perspective-correct hybrid-transparency Gaussian splatting.

The renderer itself lives in the HIP library ``libhtgs.so`` behind the C ABI
declared in ``include/htgs.h``; ``paper_2410_08129_amd.htgs`` is the thin
ctypes binding and ``torch.autograd.Function`` wrapper. Importing this package
does not load the library; the binding does, and raises if it is missing.
"""
__all__ = ["scenes", "htgs"]
