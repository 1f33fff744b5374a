"""qsv: an MI355X-native state-vector simulator core.

Submodules:
  circuits  -- seeded circuit / observable / request generators (inputs only)
  qsv       -- ctypes binding of the C-ABI library libqsv.so (HIP kernels for gfx950)
  autograd  -- adjoint-method gradient behind torch.autograd.Function
  serve     -- continuous-batching serving loop

Importing the package loads nothing native; ``paper_2604_03816_amd.qsv`` loads
libqsv.so on first use and raises if it is missing.
"""
