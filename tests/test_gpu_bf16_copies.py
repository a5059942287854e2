"""bfloat16 operand copies: the linear-layer products that read bfloat16-stored
operands give the rounding form's result bit for bit (both round each operand
to bfloat16 once, nearest even, and accumulate in the same order), and a whole
block of updates with the copies equals one without them."""
import numpy as np
import pytest
import torch

from paper_2602_21203_amd import synthetic
from tests import helpers as H

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2602_21203_amd import api


def _bf16_rows(z, rows, K, lr, gen):
    """[z, rows, K] bfloat16 view of rows lr elements long (the tail past K holds
    values that must not reach the product)."""
    full = (torch.rand((z, rows, lr), generator=gen, device="cuda") * 2 - 1).to(torch.bfloat16)
    full[..., K:] = float("nan")
    return full[..., :K]


# (batch, M, N, K, row padding past K rounded up to 8): the update's shapes (K =
# 512, 288, 274, 268, and 3872 on 32 x 32 inputs), ragged tiles, a long
# contraction and a single chunk
SHAPES = [(2, 512, 512, 512, 0), (4, 512, 512, 288, 0), (1, 1024, 256, 288, 0), (4, 512, 101, 512, 0),
          (2, 512, 512, 274, 0), (1, 1024, 512, 268, 8), (3, 33, 65, 300, 24), (2, 96, 40, 1000, 0),
          (1, 32, 32, 8, 0), (1, 7, 12, 512, 0), (2, 64, 48, 3872, 0)]


@pytest.mark.parametrize("z,M,N,K,pad", SHAPES)
def test_gemm_on_bf16_copies_equals_the_rounding_form(z, M, N, K, pad):
    print(f"gemm_bf16 z={z} M={M} N={N} K={K} pad={pad}", flush=True)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(K + 7 * M + N)
    lr = (K + 7) // 8 * 8 + pad
    A = _bf16_rows(z, M, K, lr, gen)
    B = _bf16_rows(z, N, K, lr, gen)
    bias = torch.rand((z, N), generator=gen, device="cuda")
    C1 = api.gemm_bf16(A, B, bias=bias)
    C0 = api.gemm(api.SQ_BF16, A.float(), B.float(), bias=bias)
    torch.cuda.synchronize()
    assert torch.isfinite(C1).all()
    assert torch.equal(C1, C0)
    # and the product itself, against FP64 on the same bfloat16 values
    ref = torch.matmul(A.double(), B.double().transpose(1, 2).contiguous()) + bias.double()[:, None, :]
    err = (C1.double() - ref).abs().max().item()
    scale = torch.matmul(A.double().abs(), B.double().abs().transpose(1, 2).contiguous()).max().item()
    assert err <= 1e-6 * scale, err


def test_gemm_on_bf16_copies_rejects_unaligned_rows():
    A = torch.zeros((1, 32, 12), dtype=torch.bfloat16, device="cuda")
    B = torch.zeros((1, 32, 16), dtype=torch.bfloat16, device="cuda")[..., :12]
    with pytest.raises(ValueError):
        api.gemm_bf16(A, B)


def _run(name, B, prec, copies, n_blocks=2, utd=2, eager=False):
    cfg = H.cfg(name)
    cpu = synthetic.replay(4096 if name != "full32" else 512, cfg["H"], cfg["W"], cfg["C"], cfg["proprio"],
                           cfg["action"], seed=0)
    rep = {k: (v.cuda() if torch.is_tensor(v) else v) for k, v in cpu.items()}
    was = api.bf16_operand_copies(copies)
    try:
        ag = api.Agent(cfg, H.params(name), B, prec=prec)
    finally:
        api.bf16_operand_copies(was)
    n0 = api.bf16_copy_products()
    stats = [ag.sac_update(rep, utd, graph=not eager) for _ in range(n_blocks)]
    torch.cuda.synchronize()
    return ag, torch.cat(stats).cpu().numpy(), api.bf16_copy_products() - n0


# products per update that read copies: all 22.  Forward: the input projections
# (one launch), the critics' three layers, the actor's two hidden layers and head,
# and the updated critic's four layers in the actor step.  Backward: the input and
# weight gradients of the critics' three layers and input projection and of the
# actor's three layers (one launch each), the actor's projection weight gradient,
# and in the actor step the updated critic's output and second-layer input
# gradients and the dQ/da product.  The state-based form reads its features (the
# sampled states) without a copy, so its input projections and their weight
# gradients do not; the odd widths take the general paths (counted, not pinned).
@pytest.mark.parametrize("name,B,per_update", [("tiny", 32, 22), ("full", 512, 22), ("full32", 128, 22),
                                               ("state", 512, None), ("odd", 32, None)])
def test_update_with_copies_equals_update_without(name, B, per_update):
    print(f"copies vs none {name} B={B}", flush=True)
    a1, s1, n1 = _run(name, B, 1, True)
    a0, s0, n0 = _run(name, B, 1, False)
    print(f"  products on copies: {n1} in 2 updates", flush=True)
    for attr in ("params", "target", "m", "v", "counters"):
        assert torch.equal(getattr(a1, attr), getattr(a0, attr)), attr
    np.testing.assert_array_equal(s1, s0)
    assert n0 == 0
    if per_update is not None:
        assert n1 == 2 * per_update   # counted at capture: one graph of 2 updates, replayed twice
    else:
        assert n1 > 0


def test_eager_update_counts_its_products_on_copies():
    _, s1, n1 = _run("tiny", 32, 1, True, n_blocks=1, utd=3, eager=True)
    assert n1 == 3 * 22
    assert np.all(np.isfinite(s1)) and np.all(s1[:, 7] == 0)


# transposed reads (rows contiguous, k strided): the weight-gradient form dW = dY^T X
# and the input-gradient form dX = dY W on bfloat16 copies, against the rounding form
@pytest.mark.parametrize("z,M,N,K", [(2, 512, 512, 512), (1, 256, 288, 512), (2, 512, 274, 512), (1, 64, 48, 96),
                                     (1, 40, 69, 32), (2, 33, 17, 100)])
def test_transposed_copies_equal_the_rounding_form(z, M, N, K):
    print(f"transposed z={z} M={M} N={N} K={K}", flush=True)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(M + 3 * N + K)
    r8 = lambda x: (x + 7) // 8 * 8
    # k-major storage: A^T [z][K][r8(M)], B^T [z][K][r8(N)]; the padding holds NaN
    At = (torch.rand((z, K, r8(M)), generator=gen, device="cuda") * 2 - 1).to(torch.bfloat16)
    Bt = (torch.rand((z, K, r8(N)), generator=gen, device="cuda") * 2 - 1).to(torch.bfloat16)
    At[..., M:] = float("nan")
    Bt[..., N:] = float("nan")
    A = At[..., :M].transpose(1, 2)    # [z][M][K] views, k strided
    B = Bt[..., :N].transpose(1, 2)
    C0 = api.gemm(api.SQ_BF16, A.float(), B.float())
    C1 = api.gemm_bf16(A, B)
    torch.cuda.synchronize()
    assert torch.isfinite(C1).all()
    assert torch.equal(C1, C0)
