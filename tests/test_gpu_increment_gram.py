"""Coarse increment Gram written to HBM (sigkernel_increment_gram) and the
16-bit-input option of the sweeps, against the FP64 oracle.

References for 16-bit inputs round the float32 increments to bfloat16 / half
(round to nearest even, via torch on the CPU) and sum the exact products in
double: the GPU's float32 accumulation must match them to float32 rounding."""
import numpy as np
import pytest
import torch

import oracle
import paper_2006_14794_amd as sk
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sk.load()


def rounded_increments(P, precision):
    inc = np.diff(P.astype(np.float32), axis=-2)  # float32 differences
    t = torch.from_numpy(np.ascontiguousarray(inc))
    if precision == "bf16":
        t = t.to(torch.bfloat16)
    elif precision == "f16":
        t = t.to(torch.float16)
    return t.to(torch.float64).numpy()


@pytest.mark.parametrize("precision", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("d,lx,ly", [(1, 40, 33), (3, 70, 129), (9, 256, 256), (16, 97, 65),
                                     (16, 33, 300)])
def test_gram_tiles_and_channels(precision, d, lx, ly):
    X = workloads.random_paths(100 + d, 3, lx, d)
    Y = workloads.random_paths(200 + d, 2, ly, d)
    G = sk.sigkernel_increment_gram(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(),
                                    precision=precision).cpu().numpy()
    ix, iy = rounded_increments(X, precision), rounded_increments(Y, precision)
    ref = np.einsum("apc,bqc->abpq", ix, iy)
    scale = np.einsum("apc,bqc->abpq", np.abs(ix), np.abs(iy)).max()
    assert G.shape == ref.shape
    assert np.abs(G - ref).max() <= 2e-6 * scale


@pytest.mark.parametrize("ld", [None, 256, 259, 260])
@pytest.mark.parametrize("precision", ["f32", "bf16"])
def test_row_stride_layouts(precision, ld):
    # dense rows (255 floats), rows padded to 256 floats, a stride that is
    # not a multiple of four floats and another padded multiple of four; the
    # padding columns are left untouched
    X = workloads.random_paths(400, 3, 256, 9)
    Y = workloads.random_paths(401, 2, 256, 9)
    Xc, Yc = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    out = None
    if ld is not None:
        out = torch.full((3, 2, 255, ld), -7.0, dtype=torch.float32, device="cuda")
    G = sk.sigkernel_increment_gram(Xc, Yc, precision=precision, ld=ld, out=out).cpu().numpy()
    ix, iy = rounded_increments(X, precision), rounded_increments(Y, precision)
    ref = np.einsum("apc,bqc->abpq", ix, iy)
    scale = np.einsum("apc,bqc->abpq", np.abs(ix), np.abs(iy)).max()
    assert G.shape == ref.shape
    assert np.abs(G - ref).max() <= 2e-6 * scale
    if ld is not None:
        assert torch.all(out[..., 255:] == -7.0)
    dense = sk.sigkernel_increment_gram(Xc, Yc, precision=precision).cpu().numpy()
    assert np.array_equal(dense, G)


@pytest.mark.parametrize("lx,ly", [(2, 2), (33, 5), (70, 130), (300, 34)])
def test_row_stride_ragged_tiles(lx, ly):
    # partial row blocks and partial column tiles at a padded stride
    X = workloads.random_paths(410 + lx, 2, lx, 5)
    Y = workloads.random_paths(420 + ly, 3, ly, 5)
    n = ly - 1
    ld = (n + 3) // 4 * 4 + 4
    out = torch.full((2, 3, lx - 1, ld), -7.0, dtype=torch.float32, device="cuda")
    G = sk.sigkernel_increment_gram(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(),
                                    ld=ld, out=out).cpu().numpy()
    ix, iy = rounded_increments(X, "f32"), rounded_increments(Y, "f32")
    ref = np.einsum("apc,bqc->abpq", ix, iy)
    scale = np.einsum("apc,bqc->abpq", np.abs(ix), np.abs(iy)).max()
    assert np.abs(G - ref).max() <= 2e-6 * scale
    assert torch.all(out[..., n:] == -7.0)


def test_pairs_mode_matches_oracle_gram():
    X = workloads.random_paths(7, 4, 50, 5)
    Y = workloads.random_paths(8, 4, 31, 5)
    G = sk.sigkernel_increment_gram(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(),
                                    gram=False).cpu().numpy()
    for k in range(4):
        ref = oracle.increment_gram(X[k].astype(np.float64), Y[k].astype(np.float64))
        assert np.abs(G[k] - ref).max() <= 2e-6 * np.abs(ref).max()


def test_sixteen_bit_inputs_in_the_sweep():
    # ragged pairs, d = 16, dyadic order 2: float32 inputs meet the stated
    # tolerance, 16-bit inputs cost accuracy (reported, bounded loosely here)
    xs, ys = workloads.ragged_pairs(n_pairs=48)
    X = sk.RaggedPaths.from_list(xs, "cuda")
    Y = sk.RaggedPaths.from_list(ys, "cuda")
    ref = oracle.pairs([a.astype(np.float64) for a in xs], [b.astype(np.float64) for b in ys], 2)
    errs = {}
    for prec in ("f32", "bf16", "f16"):
        got = sk.sigkernel_pair(X, Y, 2, gram_precision=prec).cpu().numpy()
        errs[prec] = float(np.max(np.abs(got - ref) / np.maximum(1.0, np.abs(ref))))
    assert errs["f32"] <= 1e-5
    assert errs["f16"] <= 2e-3 and errs["bf16"] <= 2e-2
    assert errs["bf16"] > errs["f32"]


def rounded_paths(P, precision):
    """Paths (FP64) whose increments are the 16-bit rounded ones of P."""
    inc = rounded_increments(P, precision)
    start = P[..., :1, :].astype(np.float64)
    return np.concatenate([start, start + np.cumsum(inc, axis=-2)], axis=-2)


def mixed_err(got, ref):
    return np.abs(np.asarray(got, np.float64) - ref) / np.maximum(1.0, np.abs(ref))


@pytest.mark.parametrize("precision", ["bf16", "f16"])
@pytest.mark.parametrize("d", [6, 8, 12, 16])
def test_sixteen_bit_inputs_match_rounded_paths(precision, d):
    # the sweep on 16-bit increments is the scheme on the paths with those
    # increments, to float32 rounding (d a multiple of 4 takes the increments
    # kernel with 16-byte accesses, d = 6 the one with 4-byte accesses)
    X = workloads.random_paths(300 + d, 5, 90, d)
    Y = workloads.random_paths(310 + d, 5, 70, d)
    got = sk.sigkernel_pair(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), 2,
                            gram_precision=precision).cpu().numpy()
    ref = oracle.pairs(rounded_paths(X, precision), rounded_paths(Y, precision), 2)
    assert mixed_err(got, ref).max() <= 1e-6


@pytest.mark.parametrize("precision", ["bf16", "f16"])
def test_sixteen_bit_ragged_match_rounded_paths(precision):
    xs, ys = workloads.ragged_pairs(n_pairs=24)
    X = sk.RaggedPaths.from_list(xs, "cuda")
    Y = sk.RaggedPaths.from_list(ys, "cuda")
    got = sk.sigkernel_pair(X, Y, 2, gram_precision=precision).cpu().numpy()
    ref = oracle.pairs([rounded_paths(a, precision) for a in xs],
                       [rounded_paths(b, precision) for b in ys], 2)
    assert mixed_err(got, ref).max() <= 1e-5


@pytest.mark.parametrize("precision", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("d,lx,ly", [(2, 2, 700), (7, 4, 513), (16, 66, 258), (5, 129, 257),
                                     (3, 5, 1030), (11, 200, 3)])
def test_row_blocks_and_column_chunks(precision, d, lx, ly):
    # 64-row blocks with fewer rows than waves, a last block of 1-3 rows per
    # wave, rows of several 256-column chunks with a ragged last chunk
    X = workloads.random_paths(500 + lx, 2, lx, d)
    Y = workloads.random_paths(600 + ly, 3, ly, d)
    G = sk.sigkernel_increment_gram(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(),
                                    precision=precision).cpu().numpy()
    ix, iy = rounded_increments(X, precision), rounded_increments(Y, precision)
    ref = np.einsum("apc,bqc->abpq", ix, iy)
    scale = np.einsum("apc,bqc->abpq", np.abs(ix), np.abs(iy)).max()
    assert G.shape == ref.shape
    assert np.abs(G - ref).max() <= 2e-6 * scale


@pytest.mark.parametrize("precision", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("d,lx,ly", [(17, 40, 33), (24, 70, 129), (33, 33, 300), (64, 97, 65),
                                     (40, 2, 2), (64, 258, 131)])
def test_matrix_core_channels(precision, d, lx, ly):
    # 17-64 channels go to the 32 x 32 MFMA tiles: partial row blocks, partial
    # column tiles and chunks, odd channel counts (a zero-padded last slice);
    # the bound is float32 summation of d products in any order
    X = workloads.random_paths(700 + d, 3, lx, d)
    Y = workloads.random_paths(800 + d, 2, ly, d)
    G = sk.sigkernel_increment_gram(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(),
                                    precision=precision).cpu().numpy()
    ix, iy = rounded_increments(X, precision), rounded_increments(Y, precision)
    ref = np.einsum("apc,bqc->abpq", ix, iy)
    scale = np.einsum("apc,bqc->abpq", np.abs(ix), np.abs(iy)).max()
    assert G.shape == ref.shape
    assert np.abs(G - ref).max() <= d * 2.0 ** -23 * scale


def test_matrix_core_row_stride():
    X = workloads.random_paths(900, 2, 70, 20)
    Y = workloads.random_paths(901, 3, 50, 20)
    Xc, Yc = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    out = torch.full((2, 3, 69, 53), -7.0, dtype=torch.float32, device="cuda")
    G = sk.sigkernel_increment_gram(Xc, Yc, ld=53, out=out).cpu().numpy()
    assert torch.all(out[..., 49:] == -7.0)
    assert np.array_equal(G, sk.sigkernel_increment_gram(Xc, Yc).cpu().numpy())


@pytest.mark.parametrize("d", [5, 20])
def test_pairs_mode_both_kernels(d):
    # gram=False: pair k is (x_k, y_k), on the row kernel (d <= 16) and the
    # matrix-core kernel (d > 16)
    X = workloads.random_paths(950 + d, 3, 45, d)
    Y = workloads.random_paths(960 + d, 3, 70, d)
    G = sk.sigkernel_increment_gram(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(),
                                    gram=False).cpu().numpy()
    assert G.shape == (3, 44, 69)
    ix, iy = rounded_increments(X, "f32"), rounded_increments(Y, "f32")
    ref = np.einsum("kpc,kqc->kpq", ix, iy)
    scale = np.einsum("kpc,kqc->kpq", np.abs(ix), np.abs(iy)).max()
    assert np.abs(G - ref).max() <= d * 2.0 ** -23 * scale


@pytest.mark.parametrize("d", [3, 30])
def test_one_point_paths_give_an_empty_gram(d):
    X = torch.from_numpy(workloads.random_paths(970, 2, 1, d)).cuda()
    Y = torch.from_numpy(workloads.random_paths(971, 3, 40, d)).cuda()
    G = sk.sigkernel_increment_gram(X, Y)
    assert tuple(G.shape) == (2, 3, 0, 39)
