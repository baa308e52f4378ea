"""The scene builder's BVH construction on the host (rtq_host_bvh_*, no GPU):
trees independent of the thread count, exact FP32 child bounds, leaves that
partition the primitives, and 8-bit quantized child boxes that contain the FP32
ones when decoded with the kernels' arithmetic."""
import numpy as np
import pytest

rtq = pytest.importorskip("paper_2001_02620_amd")

LEAF = 0x80000000
EMPTY = 0xFFFFFFFF


def _boxes(seed, n):
    """Random boxes with the awkward cases: duplicates, flat and point boxes,
    long thin boxes and a wide range of sizes."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-1000, 1000, size=(n, 3)) * np.array([1.0, 1.0, 0.05])
    e = np.exp(rng.uniform(np.log(1e-3), np.log(30.0), size=(n, 3)))
    e[rng.random(n) < 0.05] *= np.array([40.0, 0.01, 1.0])
    b = np.concatenate([c - e, c + e], axis=1).astype(np.float32)
    z0 = rng.random(n) < 0.02
    b[z0, 2] = b[z0, 5] = 0.0
    flat = rng.random(n) < 0.03
    b[flat, 5] = b[flat, 2]
    point = rng.random(n) < 0.01
    b[point, 3:] = b[point, :3]
    dup = np.nonzero(rng.random(n) < 0.02)[0]
    b[dup[1:]] = b[dup[:-1]]
    return b


def _leaf(c):
    return (int(c) >> 3) & 0x0FFFFFFF, (int(c) & 7) + 1


@pytest.mark.parametrize("leaf_max,bins", [(1, 64), (4, 32)])
def test_tree_does_not_depend_on_thread_count(leaf_max, bins):
    b = _boxes(1, 150_000)
    ref = rtq.host_bvh(b, leaf_max=leaf_max, bins=bins, threads=1)
    for t in (3, 8):
        r = rtq.host_bvh(b, leaf_max=leaf_max, bins=bins, threads=t)
        assert r["depth"] == ref["depth"]
        assert np.array_equal(r["order"], ref["order"])
        assert r["f32"].tobytes() == ref["f32"].tobytes(), f"FP32 nodes differ with {t} threads"
        assert r["q8"].tobytes() == ref["q8"].tobytes(), f"quantized nodes differ with {t} threads"


def _decode(q8, axis, which):
    """Decoded planes [n, 4] of one axis, lower (which=0) or upper, exactly as the
    kernels evaluate them: fmaf(q, 2^e, origin), where q 2^e is exact in FP32."""
    e = ((q8["exps"] >> (8 * axis)) & 0xFF).astype(np.int8).astype(np.int32)
    word = q8[("lo_", "hi_")[which] + "xyz"[axis]]
    q = np.stack([(word >> (8 * c)) & 0xFF for c in range(4)], axis=1).astype(np.float32)
    scale = np.ldexp(np.float32(1.0), e).astype(np.float32)[:, None]
    return (q * scale).astype(np.float32) + q8["origin"][:, axis][:, None], q


@pytest.mark.parametrize("seed,leaf_max", [(2, 4), (3, 1), (4, 8)])
def test_bounds_leaves_and_quantized_containment(seed, leaf_max):
    n = 20_000
    b = _boxes(seed, n)
    r = rtq.host_bvh(b, leaf_max=leaf_max, bins=32)
    f32, q8, order = r["f32"], r["q8"], r["order"]
    assert np.array_equal(np.sort(order), np.arange(n, dtype=np.uint32)), "leaf order is not a permutation"
    m = f32.shape[0]
    lo = np.full((m, 3), np.inf, np.float32)
    hi = np.full((m, 3), -np.inf, np.float32)
    covered = np.zeros(n, np.int32)
    # children follow their parent, so a backward sweep sees every subtree first
    for j in range(m - 1, -1, -1):
        for k in range(4):
            c = int(f32["child"][j, k])
            if c == EMPTY:
                continue
            if c & LEAF:
                first, count = _leaf(c)
                assert count <= leaf_max
                prims = order[first:first + count]
                covered[first:first + count] += 1
                clo, chi = b[prims, :3].min(axis=0), b[prims, 3:].max(axis=0)
            else:
                assert j < c < m
                clo, chi = lo[c], hi[c]
            got_lo = np.array([f32["lo_x"][j, k], f32["lo_y"][j, k], f32["lo_z"][j, k]])
            got_hi = np.array([f32["hi_x"][j, k], f32["hi_y"][j, k], f32["hi_z"][j, k]])
            # FP32 child boxes are the exact bounds of their subtrees
            assert np.array_equal(got_lo, clo) and np.array_equal(got_hi, chi), (j, k)
            lo[j] = np.minimum(lo[j], clo)
            hi[j] = np.maximum(hi[j], chi)
    assert (covered == 1).all(), "leaves do not partition the primitives"
    assert np.array_equal(q8["child"], f32["child"])
    full = f32["child"] != EMPTY
    planes = (("lo_x", "hi_x"), ("lo_y", "hi_y"), ("lo_z", "hi_z"))
    for a in range(3):
        dlo, qlo = _decode(q8, a, 0)
        dhi, qhi = _decode(q8, a, 1)
        flo, fhi = f32[planes[a][0]], f32[planes[a][1]]
        assert (dlo[full] <= flo[full]).all(), f"axis {a}: a decoded lower plane lies above the FP32 plane"
        assert (dhi[full] >= fhi[full]).all(), f"axis {a}: a decoded upper plane lies below the FP32 plane"
        assert (qlo[~full] == 255).all() and (qhi[~full] == 0).all(), "empty slots are not inverted"


def test_host_bvh_argument_errors():
    good = _boxes(5, 10)
    with pytest.raises(rtq.RtqError):
        rtq.host_bvh(good[:0])
    bad = good.copy()
    bad[3, 0] = bad[3, 3] + 1.0  # inverted
    with pytest.raises(rtq.RtqError):
        rtq.host_bvh(bad)
    bad = good.copy()
    bad[4, 5] = np.nan
    with pytest.raises(rtq.RtqError):
        rtq.host_bvh(bad)
    with pytest.raises(rtq.RtqError):
        rtq.host_bvh(good, leaf_max=9)
    with pytest.raises(rtq.RtqError):
        rtq.host_bvh(good, bins=2)
