"""MI355X-native batched LDPC decoding (binary min-sum and non-binary Min-Max).

Submodules:
  ldpcx        -- ctypes binding of the HIP library libldpcx.so (C-ABI in include/ldpcx.h)
  synth        -- seeded synthetic workloads (codes, encoders, BPSK/AWGN channel)
  build_native -- hipcc build of libldpcx.so for gfx950
"""
__all__ = ["ldpcx", "synth", "build_native"]
