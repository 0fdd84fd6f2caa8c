"""MI355X-native hot path of 3D Student Splatting and Scooping (arXiv 2503.10148).

Submodules:
  sss       -- ctypes binding of libsss.so (the C-ABI in include/sss.h)
  autograd  -- torch.autograd.Function around project/bin/render fwd+bwd
  serve     -- continuous-batching render server
  scenes    -- seeded synthetic scenes, cameras and targets (no method arithmetic)
  build     -- compiles libsss.so for gfx950

Importing the package loads nothing; the HIP library is loaded on first use
of ``paper_2503_10148_amd.sss`` and raises if it is missing.
"""
__version__ = "0.1.0"
