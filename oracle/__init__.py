"""FP64 CPU oracle for the Squint visual SAC update (arXiv 2602.21203).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy implementation of what the GPU library computes.  Only the test suite,
the smoke check and the CPU-baseline leg of the benchmark may import it.  It
shares no code with the HIP path and must never be called by the product.

Modules
  philox    Philox4x32-10 counter RNG, replay-index sampler, Box-Muller noise
  squint    area downsampling of uint8 frames
  ring      squint at insertion (uint8 block means) and the FIFO replay ring
  env       synthetic environment stub of the environment-step loop (point mass,
            integer frame renderer)
  layout    canonical flat parameter layout
  nets      conv / linear / LayerNorm / heads, forward and hand-written backward
  sac       one full SAC update (critic, temperature, actor, Adam, target EMA)
  bf16      round-to-nearest-even emulation of bfloat16 operands

Pinning status (what each function is checked against lives in tests/):
every function is pinned by an independent check except the composition of
a whole update, which the paper does not fix numerically ("parity unpinned"
for the whole-update composition; it is pinned only through its parts).
"""
