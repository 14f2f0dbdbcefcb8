"""Unit parity of the HIP kernels through the C ABI test hooks (GPU)."""

import numpy as np
import pytest

from oracle import net, philox
from tests._gpu import bf16_round, fmd_lib, normwise, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return torch_cuda(), fmd_lib()


def test_philox_bit_exact(env):
    torch, fmd = env
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2**63, size=(4096, 4), dtype=np.int64).astype(np.uint64)
    ctr[:300, 0] = np.arange(300) % 3            # the noise counters (b, slot, event, 0)
    ctr[:300, 1] = np.arange(300) // 3
    ctr[:300, 3] = 0
    ctr[-1] = [2**64 - 1] * 4
    for key in ((0, 0), (1, 0), (2**64 - 1, 2**64 - 1), (123456789, 987654321)):
        out = fmd.debug_philox(key[0], key[1], torch.from_numpy(ctr.view(np.int64)).cuda())
        got = out.cpu().numpy().view(np.uint64)
        ref = philox.philox4x64_10(ctr, np.array(key, dtype=np.uint64))
        assert np.array_equal(got, ref)


def test_noise_matches_oracle(env):
    torch, fmd = env
    off = np.array([0, 5, 5, 70, 71, 300], dtype=np.int64)      # includes an empty event
    for n_feat in (9, 4, 12):
        out = torch.zeros((off[-1], n_feat), dtype=torch.float32, device="cuda")
        fmd.noise(77, off, n_feat, out)
        torch.cuda.synchronize()
        ref = philox.noise_batch(77, off, n_feat)
        assert np.max(np.abs(out.cpu().numpy() - ref)) < 2e-5


def test_pack_padded_exact(env):
    torch, fmd = env
    rng = np.random.default_rng(1)
    E, n_max, f = 37, 50, 9
    lengths = rng.integers(0, n_max + 1, E).astype(np.int32)
    lengths[3] = 0
    lengths[4] = n_max
    padded = rng.standard_normal((E, n_max, f)).astype(np.float32)
    for e in range(E):
        padded[e, lengths[e]:] = np.nan                    # pads are never read
    off_t = torch.empty(E + 1, dtype=torch.int64, device="cuda")
    feat_t = torch.full((E * n_max, f), -7.0, dtype=torch.float32, device="cuda")
    fmd.pack_padded(torch.from_numpy(padded).cuda(), torch.from_numpy(lengths).cuda(), off_t, feat_t)
    torch.cuda.synchronize()
    off = off_t.cpu().numpy()
    assert np.array_equal(off, np.r_[0, np.cumsum(lengths)])
    ref = np.concatenate([padded[e, :lengths[e]] for e in range(E)])
    got = feat_t.cpu().numpy()[: off[-1]]
    assert np.array_equal(got, ref)
    assert np.all(feat_t.cpu().numpy()[off[-1]:] == -7.0)


def _ln(a, g, s):
    a = a.astype(np.float64)
    mu = a.mean(1, keepdims=True)
    var = ((a - mu) ** 2).mean(1, keepdims=True)
    return (a - mu) / np.sqrt(var + 1e-5) * g + s


GEMM_CASES = [  # (M, N, K, ln, epi)
    (1, 64, 64, False, 0), (130, 192, 64, True, 0), (300, 256, 256, True, 1),
    (257, 768, 256, True, 0), (129, 256, 1024, False, 2), (513, 128, 32, False, 1),
    (640, 1024, 256, True, 1), (200, 3072, 256, False, 0),
]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("M,N,K,ln,epi", GEMM_CASES)
def test_gemm(env, prec, M, N, K, ln, epi):
    torch, fmd = env
    rng = np.random.default_rng(M * 7 + N + K)
    A = (rng.standard_normal((M, K)) * 2 + 0.5).astype(np.float32)
    W = (rng.standard_normal((K, N)) / np.sqrt(K)).astype(np.float32)
    b = rng.standard_normal(N).astype(np.float32)
    g = (1 + 0.1 * rng.standard_normal(K)).astype(np.float32)
    s = (0.1 * rng.standard_normal(K)).astype(np.float32)
    C0 = rng.standard_normal((M, N)).astype(np.float32)
    dev = lambda a: torch.from_numpy(a).cuda()  # noqa: E731
    C = dev(C0.copy()) if epi == 2 else None
    out = fmd.debug_gemm(prec, dev(A), dev(W), dev(b), (dev(g), dev(s)) if ln else None, epi, C)
    torch.cuda.synchronize()
    Ap = _ln(A, g, s) if ln else A.astype(np.float64)
    Wp = W.astype(np.float64)
    if prec == 1:
        Ap = bf16_round(Ap.astype(np.float32)).astype(np.float64)
        Wp = bf16_round(W).astype(np.float64)
    ref = Ap @ Wp + b
    if epi == 1:
        ref = net.gelu(ref)
    if epi == 2:
        ref = ref + C0
    tol = 1e-5 if prec == 0 else 1.2e-2
    assert normwise(out.cpu().numpy(), ref) < tol


TILE_CASES = [  # (M, N, K, ln, epi) exercising every tiling of the autotuner
    (700, 768, 256, True, 0), (300, 1024, 256, True, 1), (513, 256, 1024, False, 2),
    (200, 256, 256, False, 2), (100, 64, 64, True, 0),
]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("M,N,K,ln,epi", TILE_CASES)
def test_gemm_every_tiling_matches(env, prec, M, N, K, ln, epi):
    """Each candidate tiling that divides the shape gives the same bits as the default."""
    torch, fmd = env
    rng = np.random.default_rng(M + N)
    dev = lambda a: torch.from_numpy(a).cuda()  # noqa: E731
    A = dev(rng.standard_normal((M, K)).astype(np.float32))
    W = dev((rng.standard_normal((K, N)) / np.sqrt(K)).astype(np.float32))
    b = dev(rng.standard_normal(N).astype(np.float32))
    g = dev((1 + 0.1 * rng.standard_normal(K)).astype(np.float32))
    s = dev((0.1 * rng.standard_normal(K)).astype(np.float32))
    C0 = rng.standard_normal((M, N)).astype(np.float32)
    ref = fmd.debug_gemm(prec, A, W, b, (g, s) if ln else None, epi,
                         dev(C0.copy()) if epi == 2 else None).cpu().numpy()
    tried = 0
    for tile in range(7):
        try:
            out = fmd.debug_gemm(prec, A, W, b, (g, s) if ln else None, epi,
                                 dev(C0.copy()) if epi == 2 else None, tile=tile).cpu().numpy()
        except fmd.FmdError as e:
            assert e.status == fmd.E_UNSUPPORTED
            continue
        tried += 1
        assert np.array_equal(out, ref), tile
    assert tried >= (1 if N < 128 else 2)


ATTN_CASES = [  # (event sizes, heads, dh)
    ([1], 1, 16), ([2, 31, 32, 33], 4, 16), ([64, 65, 1, 127, 128, 129], 8, 32),
    ([200, 3, 150], 8, 32), ([1000], 2, 32), ([17, 70], 2, 64), ([0, 5, 0, 9], 4, 32),
    ([95, 96, 97, 160, 161, 225, 255, 256, 257], 8, 32),     # 32-key group edges
    ([31, 32, 33, 63, 192, 193, 224], 8, 32),   # last chunk shortened to 32, 64 or 96 keys
]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("sizes,H,dh", ATTN_CASES)
def test_attention(env, prec, sizes, H, dh):
    torch, fmd = env
    rng = np.random.default_rng(sum(sizes) + H + dh)
    off = np.r_[0, np.cumsum(sizes)].astype(np.int64)
    T, d = int(off[-1]), H * dh
    Q, K, V = (rng.standard_normal((T, d)).astype(np.float32) * sc for sc in (1.5, 1.5, 1.0))
    dev = lambda a: torch.from_numpy(a).cuda()  # noqa: E731
    O = fmd.debug_attention(prec, off, off, H, dh, dev(Q), dev(K), dev(V))
    torch.cuda.synchronize()
    if prec == 1:
        Q, K, V = bf16_round(Q), bf16_round(K), bf16_round(V)
    ref = np.zeros((T, d))
    for e in range(len(sizes)):
        a, b = off[e], off[e + 1]
        if b > a:
            ref[a:b] = net.attention(Q[a:b].astype(np.float64), K[a:b].astype(np.float64),
                                     V[a:b].astype(np.float64), H)
    tol = 2e-6 if prec == 0 else 1.5e-2
    assert normwise(O.cpu().numpy(), ref) < tol


@pytest.mark.parametrize("prec", [0, 1])
def test_cross_attention_with_different_key_sets(env, prec):
    torch, fmd = env
    rng = np.random.default_rng(5)
    qo = np.array([0, 3, 50, 51, 251], dtype=np.int64)
    ko = np.array([0, 70, 71, 200, 233], dtype=np.int64)
    H, dh = 4, 32
    d = H * dh
    Q = rng.standard_normal((qo[-1], d)).astype(np.float32)
    K = rng.standard_normal((ko[-1], d)).astype(np.float32)
    V = rng.standard_normal((ko[-1], d)).astype(np.float32)
    dev = lambda a: torch.from_numpy(a).cuda()  # noqa: E731
    O = fmd.debug_attention(prec, qo, ko, H, dh, dev(Q), dev(K), dev(V)).cpu().numpy()
    if prec == 1:
        Q, K, V = bf16_round(Q), bf16_round(K), bf16_round(V)
    for e in range(4):
        ref = net.attention(Q[qo[e]:qo[e + 1]].astype(np.float64), K[ko[e]:ko[e + 1]].astype(np.float64),
                            V[ko[e]:ko[e + 1]].astype(np.float64), H)
        assert normwise(O[qo[e]:qo[e + 1]], ref) < (2e-6 if prec == 0 else 1.5e-2)
