"""Launch configurations of the fused iteration that the GPU tests sweep: (label groups,
tile rows, tile columns); 128 columns = two pixels per lane, which needs an even width."""
import pytest

TILINGS = [(g, t, c) for c in (64, 128) for (g, t) in ((1, 4), (1, 8), (2, 4), (2, 8), (4, 4))] + [(1, 2, 64)]
TILING_IDS = [f"g{g}t{t}c{c}" for g, t, c in TILINGS]


LDS_PER_WORKGROUP = 160 * 1024   # MI355X (gfx950)


def lds_bytes(tiling, k: int) -> int:
    """LDS a workgroup of the fused iteration needs: the sbar and s planes of every label
    for the tile's pixels, the chunk sums and the straddle results."""
    g, t, c = tiling
    npx = t * c
    reg = c == 64 and g == 1
    return 4 * (2 * k * npx + g * npx + (2 if reg else 4 * npx))


def use_tiling(prob, tiling, width: int, k: int = 1) -> bool:
    """Apply `tiling` to a problem; for pixel pairs on an odd width, or a tiling whose LDS
    does not fit a workgroup at k labels, check that the library rejects it
    (SL_ERR_UNSUPPORTED) and return False."""
    import paper_1512_01383_amd as S
    if (tiling[2] == 128 and width % 2) or lds_bytes(tiling, k) > LDS_PER_WORKGROUP:
        with pytest.raises(S.SublabelError) as e:
            prob.set_tiling(*tiling)
        assert e.value.status == 2
        return False
    prob.set_tiling(*tiling)
    assert prob.get_tiling() == tuple(tiling)
    return True
