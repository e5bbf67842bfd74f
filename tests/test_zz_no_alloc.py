"""ej_verify_static, the verification entry point that allocates no device
memory (its workspace is a static device array), against ej_verify on the same
inputs: bit-exact distances on two calls in a row, the second with a smaller
input, per-pair thresholds, every verification form, and the refusal of an
input whose workspace exceeds the array."""
import sys

import numpy as np
import pytest

import synthdata as sd

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ej():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1702_00093_amd as ej
    ej.lib()
    return ej


def _pairs(rng, n, count):
    a = rng.integers(0, n, size=count)
    b = rng.integers(0, n, size=count)
    return (a.astype(np.uint64) << np.uint64(32)) | b.astype(np.uint64)


def _device(col, codes):
    import torch
    chars = torch.from_numpy(col.chars.copy()).cuda()
    offs = torch.from_numpy(col.offsets.astype(np.int64)).cuda()
    pairs = torch.from_numpy(codes.astype(np.int64)).cuda()
    return chars, offs, pairs


def test_static_verify_equals_verify_twice_second_smaller(ej, oracle_lib):
    import torch
    rng = np.random.default_rng(11)
    big = sd.clusters(301, 40, lambda rr, b: 5, lambda rr: rr.integers(800, 3000),
                      lambda rr, LL: rr.poisson(0.03 * LL))
    small = sd.clusters(302, 6, lambda rr, b: 3, lambda rr: rr.integers(50, 400),
                        lambda rr, LL: rr.poisson(5))
    fresh = ej.Context(0)  # nothing allocated yet: the call must leave it so
    ref_ctx = ej.Context(0)
    try:
        for step, (col, K, count) in enumerate([(big, 120, 3000), (small, 30, 200)]):
            codes = _pairs(rng, col.n, count)
            chars, offs, pairs = _device(col, codes)
            want = ref_ctx.verify(chars, offs, pairs, K).cpu().numpy()
            dist = torch.full((count,), -7, dtype=torch.int32, device="cuda")
            _say(f"verify_static call {step}: n={col.n} pairs={count} K={K}")
            got = fresh.verify(chars, offs, pairs, K, dist=dist, no_alloc=True).cpu().numpy()
            assert got.tolist() == want.tolist()
            assert fresh.workspace_bytes == 0
            # and both equal the oracle on a sample
            idx = rng.choice(count, size=min(count, 150), replace=False)
            o = oracle_lib.verify_pairs(col.chars, col.offsets, codes[idx], K)
            assert got[idx].astype(np.uint32).tolist() == o.tolist()
    finally:
        fresh.close()
        ref_ctx.close()


def test_static_verify_every_form_and_per_pair_thresholds(ej, oracle_lib):
    import torch
    rng = np.random.default_rng(12)
    col = sd.clusters(303, 12, lambda rr, b: 4, lambda rr: rr.integers(100, 1500),
                      lambda rr, LL: rr.poisson(40))
    codes = _pairs(rng, col.n, 400)
    Kq = rng.integers(0, 600, size=400).astype(np.int32)
    chars, offs, pairs = _device(col, codes)
    dKq = torch.from_numpy(Kq).cuda()
    ctx = ej.Context(0)
    try:
        for mode in (0, 1, 2, 3):
            ctx.tune_set("verify_mode", mode)
            for K, kq in ((300, None), (0, dKq)):
                want = ctx.verify(chars, offs, pairs, K, d_Kq=kq).cpu().numpy()
                _say(f"verify_static mode={mode} per-pair={kq is not None}")
                got = ctx.verify(chars, offs, pairs, K, d_Kq=kq, no_alloc=True).cpu().numpy()
                assert got.tolist() == want.tolist()
            assert ctx.tune_get("verify_mode") == mode  # the call restores the knob
    finally:
        ctx.close()


def test_static_verify_refuses_inputs_beyond_the_array(ej):
    import torch
    # 80 MB of text: its codes alone exceed the 64 MiB array
    n, ln = 20, 4_000_000
    chars = torch.from_numpy(np.tile(np.frombuffer(b"ACGT", np.uint8), n * ln // 4).copy()).cuda()
    offs = torch.arange(0, n * ln + 1, ln, dtype=torch.int64).cuda()
    pairs = torch.tensor([(0 << 32) | 1], dtype=torch.int64).cuda()
    dist = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    ctx = ej.Context(0)
    try:
        _say("verify_static beyond the scratch size")
        with pytest.raises(ej.EmbedJoinError) as ei:
            ctx.verify(chars, offs, pairs, 10, dist=dist, no_alloc=True)
        assert ei.value.status == ej.EJ_ENOMEM and "static scratch" in str(ei.value)
        assert int(dist[0]) == -7  # nothing written
        # the context still works afterwards, with and without the array
        small = torch.tensor([(0 << 32) | 1], dtype=torch.int64).cuda()
        c2 = torch.from_numpy(np.frombuffer(b"ACGTACGTAC", np.uint8).copy()).cuda()
        o2 = torch.tensor([0, 5, 10], dtype=torch.int64).cuda()
        # "ACGTA" and "CGTAC": one deletion and one insertion
        assert ctx.verify(c2, o2, small, 2, no_alloc=True).cpu().tolist() == [2]
        assert ctx.verify(c2, o2, small, 2).cpu().tolist() == [2]
        assert ctx.verify(c2, o2, small, 1, no_alloc=True).cpu().tolist() == [2]
    finally:
        ctx.close()
