"""MI355X (gfx950) set-intersection engine for triangle and 4-clique counting.

Reimplements the hot path of EmptyHeaded (Aberger et al., SIGMOD 2016): the
set intersections inside Generic-Join over a degree-ordered two-level trie.

Submodules:
  eh      -- ctypes binding of the C ABI in include/eh.h (the product path)
  inputs  -- seeded synthetic graph and request generators
  build   -- compiles the HIP library for gfx950
  autotune -- searches the performance knobs of a workload
"""
__all__ = ["eh", "inputs", "build"]
