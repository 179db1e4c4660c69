"""MI355X-native batched TFHE gate bootstrapping (the hot path under
CryptoEmu's homomorphic functional units, arXiv 2101.03403).

Modules:
  cemu       -- ctypes binding of libcemu.so (C ABI in include/cemu.h)
  circuits   -- gate-level circuits (Kogge-Stone ADD/SUB, ...) and the level
                scheduler that batches each circuit level into one launch
  workloads  -- seeded synthetic inputs (no cryptographic arithmetic)
  build      -- builds libcemu.so for gfx950
"""
