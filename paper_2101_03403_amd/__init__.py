"""MI355X-native batched TFHE gate bootstrapping (the hot path under
CryptoEmu's homomorphic functional units, arXiv 2101.03403).

Modules:
  cemu       -- ctypes binding of libcemu.so (C ABI in include/cemu.h)
  circuits   -- gate-level circuits of the functional units (Kogge-Stone
                ADD/SUB, compare, bitwise, array and sequential multipliers,
                divider, barrel shifters, NZCV flags) and the level scheduler
                that batches each circuit level into one launch
  emulator   -- the instruction-set front-end: encrypted registers and data
                memory, cleartext PC, client-resolved branches
  autotune   -- per-width choice of product form and launch shape
  workloads  -- seeded synthetic inputs (no cryptographic arithmetic)
  build      -- builds libcemu.so for gfx950
"""
