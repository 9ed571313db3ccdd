"""MI355X-native (gfx950) MPDP join-order optimizer.

  workloads   seeded synthetic join graphs (no optimizer arithmetic)
  mpdp        ctypes binding of the C-ABI in include/mpdp.h (libmpdp.so)
  build       hipcc build of libmpdp.so from csrc/

Importing the package loads nothing; ``paper_2202_13511_amd.mpdp.load()``
loads the HIP library and fails loudly when it has not been built.
"""
__all__ = ["workloads", "mpdp", "build"]
