"""Host-side checks of the motion-correction ABI (no GPU needed)."""
import pytest

from paper_2403_16438_amd import abi


def test_default_config_and_workspace():
    c = abi.seg_mc_default_config(256, 256)
    assert (c.height, c.width, c.radius) == (256, 256, 8)
    n = abi.seg_mc_workspace_bytes(c)
    # template, two integral images, two window tables, 8 slices x 2048 frames x 304 vectors
    assert n >= 256 * 256 * 2 + 2 * 257 * 257 * 8 + 2 * 121 * 304 * 8 + 8 * 2048 * 304 * 8


@pytest.mark.parametrize("h,w,r", [(256, 256, 0), (256, 256, 11), (36, 256, 8), (256, 36, 8),
                                   (4096, 64, 2), (22, 22, 1)])
def test_invalid_configs(h, w, r):
    c = abi.seg_mc_config(height=h, width=w, radius=r)
    with pytest.raises(abi.SegError) as e:
        abi.seg_mc_workspace_bytes(c)
    assert e.value.code == abi.SEG_E_INVAL


def test_smallest_frames_accepted():
    for r in (1, 5, 10):
        c = abi.seg_mc_config(height=21 + 2 * r, width=21 + 2 * r, radius=r)
        assert abi.seg_mc_workspace_bytes(c) > 0


def test_null_arguments():
    assert abi.lib.seg_mc_default_config(8, 8, None) == abi.SEG_E_INVAL
    assert abi.lib.seg_mc_create(None, None, 0, None) == abi.SEG_E_INVAL
    assert abi.lib.seg_mc_estimate(None, None, 0, None, None, None) == abi.SEG_E_INVAL
    assert abi.lib.seg_mc_apply(None, None, 0, None, None, None) == abi.SEG_E_INVAL
    assert abi.lib.seg_mc_destroy(None) == abi.SEG_OK
