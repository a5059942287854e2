"""Workload configurations (network dims + data geometry) used by tests and the benchmark.

tiny   32x32x3 frames squinted 2x to 16x16; 2 convs of 16 channels; projection 64;
       critics / actor 64-64; 51 atoms on [-10, 10]
full   64x64x9 frames (stack of 3 RGB) squinted 4x; 3 convs of 32 channels; projection 256;
       critics / actor 512-512; 101 atoms on [-20, 20]
full128  the full network on 128x128x9 frames squinted 8x
full32   the full network on 128x128x9 frames squinted 4x to 32x32 (the higher-resolution
         variant of Sec. VI Camera Resolution Analysis): convs 32 -> 15 -> 13 -> 11
state, state_tiny   state-based SAC (Sec. VI Generality and Timing Analysis): no image
         and no encoder, a 40-float state vector feeds the projections
odd      the tiny geometry with widths off the kernels' tiles (projection 40, hidden 48,
         action 17)
"""
TINY = dict(C=3, H=32, W=32, k=2, n_conv=2, F=16, proj=64, hidden=64, atoms=51, proprio=12, action=6,
            v_min=-10.0, v_max=10.0)
FULL = dict(C=9, H=64, W=64, k=4, n_conv=3, F=32, proj=256, hidden=512, atoms=101, proprio=12, action=6,
            v_min=-20.0, v_max=20.0)
FULL128 = dict(FULL, H=128, W=128, k=8)
FULL32 = dict(FULL, H=128, W=128, k=4)
# state-based SAC (no image, no encoder): a 40-float state vector in place of the
# features; the frame fields only size the (unused) frames of the synthetic replay
STATE_TINY = dict(TINY, n_conv=0, H=8, W=8, k=1, proprio=40)
STATE = dict(FULL, n_conv=0, H=8, W=8, C=3, k=1, proprio=40)
# widths that are not multiples of the kernels' tiles (projection 40, hidden 48,
# a 17-dimensional action, so the policy head spans two GEMM column tiles): the
# paths for general shapes
ODD = dict(TINY, proj=40, hidden=48, action=17)
CONFIGS = dict(tiny=TINY, full=FULL, full128=FULL128, full32=FULL32, state_tiny=STATE_TINY, state=STATE, odd=ODD)
