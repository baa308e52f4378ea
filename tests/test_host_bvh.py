"""The scene builder's BVH construction on the host (rtq_host_bvh_*, no GPU), at
node widths 2, 4 and 8: trees independent of the thread count, exact FP32 child
bounds, leaves that partition the primitives, and 8-bit quantized child boxes
that contain the FP32 ones when decoded with the kernels' arithmetic."""
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


@pytest.mark.parametrize("leaf_max,bins,width", [(1, 64, 4), (4, 32, 4), (4, 32, 8), (2, 32, 2)])
def test_tree_does_not_depend_on_thread_count(leaf_max, bins, width):
    b = _boxes(1, 150_000)
    ref = rtq.host_bvh(b, leaf_max=leaf_max, bins=bins, threads=1, width=width)
    for t in (3, 8):
        r = rtq.host_bvh(b, leaf_max=leaf_max, bins=bins, threads=t, width=width)
        assert r["depth"] == ref["depth"]
        assert np.array_equal(r["order"], ref["order"])
        assert r["wide"].tobytes() == ref["wide"].tobytes(), f"nodes differ with {t} threads"
        assert r["q8"].tobytes() == ref["q8"].tobytes(), f"quantized nodes differ with {t} threads"


def _q8_planes(q8, width, axis, which):
    """Byte planes [n, width] of one axis, lower (which=0) or upper, in each
    width's layout."""
    if width == 4:
        word = q8[("lo_", "hi_")[which] + "xyz"[axis]]
        return np.stack([(word >> (8 * c)) & 0xFF for c in range(4)], axis=1)
    if width == 8:
        w2 = q8[("lo_", "hi_")[which] + "xyz"[axis]]
        return np.stack([(w2[:, c // 4] >> (8 * (c % 4))) & 0xFF for c in range(8)], axis=1)
    word = q8["xyz"[axis]]
    return np.stack([(word >> (8 * (2 * which + c))) & 0xFF for c in range(2)], axis=1)


def _decode(q8, width, axis, which):
    """Decoded planes [n, width] of one axis exactly as the kernels evaluate them:
    fmaf(q, 2^e, origin), where q 2^e is exact in FP32."""
    e = ((q8["exps"] >> (8 * axis)) & 0xFF).astype(np.int8).astype(np.int32)
    q = _q8_planes(q8, width, axis, which).astype(np.float32)
    scale = np.ldexp(np.float32(1.0), e).astype(np.float32)[:, None]
    return (q * scale).astype(np.float32) + q8["origin"][:, axis][:, None], q


@pytest.mark.parametrize("seed,leaf_max,width", [(2, 4, 4), (3, 1, 4), (4, 8, 4), (5, 4, 8), (6, 1, 8), (7, 4, 2)])
def test_bounds_leaves_and_quantized_containment(seed, leaf_max, width):
    n = 20_000
    b = _boxes(seed, n)
    r = rtq.host_bvh(b, leaf_max=leaf_max, bins=32, width=width)
    wide, q8, order = r["wide"], r["q8"], r["order"]
    assert np.array_equal(np.sort(order), np.arange(n, dtype=np.uint32)), "leaf order is not a permutation"
    m = wide.shape[0]
    assert (wide["child"][:, width:] == EMPTY).all(), "slots beyond the width are used"
    lo = np.full((m, 3), np.inf, np.float32)
    hi = np.full((m, 3), -np.inf, np.float32)
    covered = np.zeros(n, np.int32)
    n_children = 0
    # children follow their parent, so a backward sweep sees every subtree first
    for j in range(m - 1, -1, -1):
        for k in range(width):
            c = int(wide["child"][j, k])
            if c == EMPTY:
                continue
            n_children += 1
            if c & LEAF:
                first, count = _leaf(c)
                assert count <= leaf_max
                prims = order[first:first + count]
                covered[first:first + count] += 1
                clo, chi = b[prims, :3].min(axis=0), b[prims, 3:].max(axis=0)
            else:
                assert j < c < m
                clo, chi = lo[c], hi[c]
            # FP32 child boxes are the exact bounds of their subtrees
            assert np.array_equal(wide["lo"][j, :, k], clo) and np.array_equal(wide["hi"][j, :, k], chi), (j, k)
            lo[j] = np.minimum(lo[j], clo)
            hi[j] = np.maximum(hi[j], chi)
    assert (covered == 1).all(), "leaves do not partition the primitives"
    # the greedy collapse fills more than half of every node's slots on
    # average (measured: 2.0 of 2, 3.07 of 4, 4.2 of 8)
    assert n_children / m > 0.5 * width, (n_children / m, width)
    assert np.array_equal(q8["child"], wide["child"][:, :width])
    if width == 4:
        f32 = r["f32"]
        for a, ax in enumerate("xyz"):
            assert np.array_equal(f32["lo_" + ax], wide["lo"][:, a, :4])
            assert np.array_equal(f32["hi_" + ax], wide["hi"][:, a, :4])
        assert np.array_equal(f32["child"], wide["child"][:, :4])
    else:
        assert r["f32"] is None
    full = wide["child"][:, :width] != EMPTY
    for a in range(3):
        dlo, qlo = _decode(q8, width, a, 0)
        dhi, qhi = _decode(q8, width, a, 1)
        flo, fhi = wide["lo"][:, a, :width], wide["hi"][:, a, :width]
        assert (dlo[full] <= flo[full]).all(), f"axis {a}: a decoded lower plane lies above the FP32 plane"
        assert (dhi[full] >= fhi[full]).all(), f"axis {a}: a decoded upper plane lies below the FP32 plane"
        assert (qlo[~full] == 255).all() and (qhi[~full] == 0).all(), "empty slots are not inverted"


def test_wider_nodes_make_shallower_trees():
    b = _boxes(8, 50_000)
    d = {w: rtq.host_bvh(b, leaf_max=4, bins=32, width=w)["depth"] for w in (2, 4, 8)}
    assert d[2] > d[4] > d[8], d


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
    with pytest.raises(rtq.RtqError):
        rtq.host_bvh(good, width=3)
