"""cc_gemm_noalloc (the allocation-free product) against cc_diag_gemm_batched,
the entry point it is a variant of: same kernels, same split-K chunks, so
the results must be bitwise equal. Each case runs two calls in a row, the
second on a smaller product, so the second reads a scratch array that still
holds the first call's contents. A product whose rounded operand copies do
not fit the fixed array is refused before any work is queued.
"""

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    import paper_2608_06669_amd as pk
    pk.load()
    assert torch.cuda.is_available(), "a GPU is required"
    return pk


# (M, N, K, nbatch, precision, precast, split-K, transpose A)
CASES = [
    (100, 90, 4096, 1, "fp64", False, True, False),     # split into chunks
    (64, 70, 1024, 3, "fp64", False, True, True),       # batched split-K, A transposed
    (1024, 1030, 300, 2, "bf16", True, False, False),   # operands rounded once into the array
    (2100, 2100, 512, 1, "fp32", True, True, True),     # 128 x 128 tiles, rounded operands
    (200, 300, 2048, 1, "bf16", True, True, False),     # split-K and rounded operands together
]


def _operands(M, N, K, nb, ta, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    A = torch.randn(nb, K, M, generator=g, dtype=torch.float64) if ta else \
        torch.randn(nb, M, K, generator=g, dtype=torch.float64)
    B = torch.randn(nb, K, N, generator=g, dtype=torch.float64)
    C0 = torch.randn(nb, M, N, generator=g, dtype=torch.float64)
    a_str = (1, M, M * K) if ta else (K, 1, M * K)
    return A.cuda(), B.cuda(), C0.cuda(), a_str, (N, 1, N * K), (N, 1, M * N)


@pytest.mark.parametrize("case", CASES)
def test_noalloc_product_equals_the_allocating_one(lib, case):
    M, N, K, nb, prec, pre, sk, ta = case
    for k, (m, n, kk) in enumerate([(M, N, K), (max(1, M // 2 - 3), max(1, N // 2 + 1), max(1, K // 2 - 5))]):
        A, B, C0, a_str, b_str, c_str = _operands(m, n, kk, nb, ta, 1000 * k + m + n + kk)
        ref = C0.clone()
        lib.diag_gemm_batched(A, B, ref, a_str, b_str, c_str, m, n, kk, nb, alpha=0.75, beta=-0.5, prec=prec,
                              precast=pre, splitk=sk)
        got = C0.clone()
        lib.gemm_noalloc(A, B, got, a_str, b_str, c_str, m, n, kk, nb, alpha=0.75, beta=-0.5, prec=prec,
                         precast=pre, splitk=sk)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (k, (got - ref).abs().max().item())
        # and the product is right (float64 reference, loose for FP32/BF16)
        Am = A.transpose(1, 2) if ta else A
        exact = 0.75 * torch.bmm(Am.contiguous(), B) - 0.5 * C0
        tol = {"fp64": 1e-12, "fp32": 1e-4, "bf16": 5e-2}[prec] * kk ** 0.5
        assert (got - exact).abs().max().item() <= tol, k


def test_noalloc_refuses_operand_copies_beyond_the_array(lib):
    """BF16 operand copies of nbatch (M + N) K = 16384 * 1024 elements need
    32 MiB plus alignment, above the 32 MiB part of the array: CC_ERR_OOM,
    and nothing is written."""
    A = torch.zeros(4, device="cuda", dtype=torch.float64)
    C = torch.full((4,), 3.0, device="cuda", dtype=torch.float64)
    with pytest.raises(lib.CCError) as err:
        lib.gemm_noalloc(A, A, C, (1024, 1, 0), (8192, 1, 0), (8192, 1, 0), 8192, 8192, 1024, 1, prec="bf16",
                         precast=True)
    assert err.value.status == -2  # CC_ERR_OOM
    torch.cuda.synchronize()
    assert torch.equal(C, torch.full((4,), 3.0, device="cuda", dtype=torch.float64))
