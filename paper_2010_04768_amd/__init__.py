"""MI355X-native IP-GFCCSD linear-solve path (arXiv 2010.04768).

The product is the C-ABI library ``libgfcc.so`` (HIP kernels for gfx950,
declared in ``include/gfcc.h``); ``paper_2010_04768_amd.gfcc`` is its ctypes
binding.  Importing the package loads nothing.
"""
