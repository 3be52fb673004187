"""MI355X-native ML-CG ptychography: HIP kernels behind a C ABI (libptyg.so)
with a thin ctypes binding.  Importing the package loads nothing; the HIP
library is loaded on first use by `paper_2106_07575_amd.ptyg`."""
__all__ = ["synth"]
