"""MI355X (gfx950) Gaussian ray tracer: LBVH over per-Gaussian unit-sphere instances,
multi-round k-buffer tracing with traversal checkpointing, front-to-back blending.

Submodules:
  grtx    -- ctypes binding of libgrtx.so (the C ABI in include/grtx.h); needs torch.
  inputs  -- seeded synthetic scenes, cameras and rays (numpy only).
  build   -- compiles libgrtx.so with hipcc for gfx950.
"""
