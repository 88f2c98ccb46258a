"""hr_hybrid_loss_noalloc (library-owned static scratch, no allocation)
against hr_hybrid_loss with a caller scratch buffer, through the C ABI.

Two calls in a row, the second on fewer and smaller images, so the static
array holds the first call's contents when the second runs; every output
must equal the buffered entry point's bit for bit (same kernels, same
deterministic reduction order)."""
import ctypes as C

import numpy as np
import pytest

from helpers import say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _inputs(rng, sizes):
    parts = {k: [] for k in ("image", "T", "mesh", "tri", "target")}
    for (w, h) in sizes:
        parts["image"].append(rng.uniform(0, 1, (3, h, w)).astype(np.float32))
        parts["T"].append(rng.uniform(0, 1, (h, w)).astype(np.float32))
        parts["mesh"].append(rng.uniform(0, 1, (3, h, w)).astype(np.float32))
        parts["tri"].append(np.where(rng.uniform(size=(h, w)) < 0.6, 3, -1).astype(np.int32))
        parts["target"].append(rng.uniform(0, 1, (3, h, w)).astype(np.float32))
    return {k: torch.as_tensor(np.concatenate([x.reshape(-1) for x in v])).cuda()
            for k, v in parts.items()}


def _outs(x):
    return (torch.zeros(1, dtype=torch.float32, device="cuda"), torch.empty_like(x["image"]),
            torch.empty_like(x["T"]), torch.empty_like(x["mesh"]))


def _call(hr, x, sizes, noalloc, detach=False):
    L = hr.load()
    loss, gi, gt, gm = _outs(x)
    sz = hr._sizes_array(sizes)
    flags = hr.HR_FLAG_DETACH_MASK if detach else 0
    p = hr._ptr
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if noalloc:
        rc = L.hr_hybrid_loss_noalloc(p(x["image"]), p(x["T"]), p(x["mesh"]), p(x["tri"]),
                                      p(x["target"]), sz, len(sizes), 0.1, 20.0, flags, p(loss),
                                      p(gi), p(gt), p(gm), st)
    else:
        scratch = torch.empty(hr.loss_scratch_bytes(sizes), dtype=torch.uint8, device="cuda")
        rc = L.hr_hybrid_loss(p(x["image"]), p(x["T"]), p(x["mesh"]), p(x["tri"]),
                              p(x["target"]), sz, len(sizes), 0.1, 20.0, flags, p(loss), p(gi),
                              p(gt), p(gm), p(scratch), st)
    hr.check(rc)
    torch.cuda.synchronize()
    return loss, gi, gt, gm


def test_noalloc_loss_equals_buffered_loss_on_two_calls(hr):
    rng = np.random.default_rng(12)
    for sizes, detach in (([(640, 480), (37, 29), (1280, 720)], False),
                          ([(64, 48), (5, 70)], True)):
        say(f"case: noalloc loss, sizes {sizes}, detach {detach}")
        x = _inputs(rng, sizes)
        a = _call(hr, x, sizes, noalloc=True, detach=detach)
        b = _call(hr, x, sizes, noalloc=False, detach=detach)
        for u, v in zip(a, b):
            assert torch.equal(u, v)


def test_noalloc_loss_rejects_inputs_beyond_its_limit(hr):
    L = hr.load()
    big = [(8192, 8192), (1, 1)]  # 2^26 + 1 pixels
    sz = hr._sizes_array(big)
    rc = L.hr_hybrid_loss_noalloc(4096, 4096, 4096, 4096, 4096, sz, 2, 0.1, 20.0, 0, 4096, 4096,
                                  4096, 4096, None)
    assert rc == hr.HR_ERR_INVALID_ARGUMENT and b"at most" in L.hr_last_error()
    many = hr._sizes_array([(1, 1)] * 257)
    rc = L.hr_hybrid_loss_noalloc(4096, 4096, 4096, 4096, 4096, many, 257, 0.1, 20.0, 0, 4096,
                                  4096, 4096, 4096, None)
    assert rc == hr.HR_ERR_INVALID_ARGUMENT
