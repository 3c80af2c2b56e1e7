"""Host-side scheduling for crowded fields: the source colouring of celeste_colour_sources
(no GPU work) and batch subsets."""
import numpy as np

import synth


def _boxes(sb):
    out = []
    for s in range(sb.n_sources):
        i0, i1 = sb.src_img_off[s], sb.src_img_off[s + 1]
        ox, oy = sb.img_origin[i0:i1, 0], sb.img_origin[i0:i1, 1]
        out.append((ox.min(), (ox + sb.img_w[i0:i1]).max(), oy.min(), (oy + sb.img_h[i0:i1]).max()))
    return out


def _hit(a, b):
    return a[0] < b[1] and b[0] < a[1] and a[2] < b[3] and b[2] < a[3]


def test_colouring_is_conflict_free_and_greedy():
    from paper_1611_03404_amd import celeste as cb
    sf = synth.make_field(n_sources=400, size=256, epochs=1, seed=5)
    sb = sf.batch
    col, n = cb.colour_sources(cb.Batch.from_synth(sb))
    assert col.min() == 0 and col.max() == n - 1
    box = _boxes(sb)
    # no two sources of one colour share a pixel of any field image
    for c in range(n):
        members = np.nonzero(col == c)[0]
        for a in range(len(members)):
            for b in range(a + 1, len(members)):
                s, t = members[a], members[b]
                for i in range(sb.src_img_off[s], sb.src_img_off[s + 1]):
                    for j in range(sb.src_img_off[t], sb.src_img_off[t + 1]):
                        if sf.img_field[i] != sf.img_field[j]:
                            continue
                        ri = (sb.img_origin[i, 0], sb.img_origin[i, 0] + sb.img_w[i],
                              sb.img_origin[i, 1], sb.img_origin[i, 1] + sb.img_h[i])
                        rj = (sb.img_origin[j, 0], sb.img_origin[j, 0] + sb.img_w[j],
                              sb.img_origin[j, 1], sb.img_origin[j, 1] + sb.img_h[j])
                        assert not _hit(ri, rj), (s, t, i, j)
    # greedy in source order: every smaller colour is taken by an earlier overlapping source
    for s in range(sb.n_sources):
        taken = {int(col[t]) for t in range(s) if _hit(box[s], box[t])}
        assert int(col[s]) not in taken
        assert all(c in taken for c in range(int(col[s])))
    # a field holding one source needs one colour
    one = sb.subset([3])
    c1, n1 = cb.colour_sources(cb.Batch.from_synth(one))
    assert n1 == 1 and c1[0] == 0


def test_subset_batch_shares_images():
    from paper_1611_03404_amd import celeste as cb
    sb = synth.make_config(1, n_sources=7)
    b = cb.Batch.from_synth(sb)
    sub, img_idx = b.subset([5, 1, 2])
    assert sub.n_sources == 3
    want = np.concatenate([np.arange(sb.src_img_off[s], sb.src_img_off[s + 1]) for s in (5, 1, 2)])
    assert np.array_equal(img_idx, want)
    assert np.array_equal(sub.images, b.images[want])
    assert np.array_equal(sub.offsets, [0, 5, 10, 15])
