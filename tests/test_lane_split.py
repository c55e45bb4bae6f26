"""The gravity kernels split a 256-lane workgroup over tc targets without
integer division: G = trunc((256 + 1/2) r), g = trunc((tid + 1/2) r) with
r an FP32 reciprocal of tc accurate to one ulp.  Emulated here in FP32 with
the reciprocal off by up to two ulps either way: every quotient is exact."""
import numpy as np


def test_float_lane_split_is_exact():
    v = np.arange(0, 257, dtype=np.float32)
    want_all = np.arange(0, 257)
    for tc in range(1, 257):
        r0 = np.float32(1.0) / np.float32(tc)
        for ulps in (-2, -1, 0, 1, 2):
            r = r0
            for _ in range(abs(ulps)):
                r = np.nextafter(r, np.float32(np.inf if ulps > 0 else 0), dtype=np.float32)
            q = ((v + np.float32(0.5)) * r).astype(np.float32)
            got = q.astype(np.int64)                      # truncation, as the kernel's cast
            np.testing.assert_array_equal(got, want_all // tc)


def test_component_reduction_covers_every_target_once():
    # With 4 tc <= 256 the partial sums are reduced by lane (t, g), g < 4, one
    # per (target, component): every pair (t, c) has exactly one such lane, that
    # lane is active (g < G), and the partials it reads, lanes q tc + t for
    # q < G, are all active lanes.  Wider chunks leave the sums to lanes t < tc.
    tid = np.arange(256)
    for tc in range(1, 257):
        G = 256 // tc
        g, t = tid // tc, tid % tc
        if 4 * tc <= 256:
            sel = g < 4
            assert np.all(g[sel] < G)
            pairs = set(zip(t[sel].tolist(), g[sel].tolist()))
            assert len(pairs) == sel.sum() == 4 * tc
            assert pairs == {(a, c) for a in range(tc) for c in range(4)}
        reads = (np.arange(G)[:, None] * tc + np.arange(tc)[None, :]).ravel()
        assert reads.max() < G * tc <= 256
        assert np.all(reads // tc < G)
