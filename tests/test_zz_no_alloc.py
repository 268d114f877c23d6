"""The allocation-free entry point (ddgs_sort_pairs_noalloc) against the
allocating one it mirrors (ddgs_debug_sort_pairs), through the C ABI: two
calls in a row, the second with a smaller input, bit-identical results, no
workspace allocation, and the size limit."""
import numpy as np
import pytest

from paper_2406_02518_amd import binding

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_noalloc_sort_matches_the_allocating_sort():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    R = binding.Renderer(0)
    try:
        rng = np.random.default_rng(71)
        for n, bits in ((1 << 20, 32), (300001, 21)):
            keys = rng.integers(0, 1 << bits, size=n, dtype=np.uint64).astype(np.uint32)
            keys[::7] = keys[3]  # many equal keys: stability matters
            vals = rng.permutation(n).astype(np.uint32)
            ka, va = torch.from_numpy(keys).cuda(), torch.from_numpy(vals).cuda()
            kb, vb = ka.clone(), va.clone()
            binding.ddgs_debug_sort_pairs(R.ctx, ka.data_ptr(), va.data_ptr(), n, bits)
            held = R.allocator.bytes_held()
            with torch.cuda.stream(R.stream):
                binding.ddgs_sort_pairs_noalloc(R.ctx, kb.data_ptr(), vb.data_ptr(), n, bits)
            R.stream.synchronize()
            assert R.allocator.bytes_held() == held  # the workspace was not touched
            np.testing.assert_array_equal(kb.cpu().numpy(), ka.cpu().numpy())
            np.testing.assert_array_equal(vb.cpu().numpy(), va.cpu().numpy())
            order = np.argsort(keys, kind="stable")
            np.testing.assert_array_equal(kb.cpu().numpy(), keys[order])
            np.testing.assert_array_equal(vb.cpu().numpy(), vals[order])
        big = torch.zeros((1 << 20) + 1, dtype=torch.int32, device="cuda")
        with pytest.raises(binding.DDGSError, match="static scratch limit"):
            binding.ddgs_sort_pairs_noalloc(R.ctx, big.data_ptr(), big.data_ptr(), big.numel(), 32)
    finally:
        R.close()
