"""Per-component NMF at ranks 3 to 8 (Eq. 3) on both execution paths.

One component holds n overlapping cells, each spiking alone in some
segments, so the successive projection finds rank n (the HALS loop is
compiled per rank). The GPU's footprints against the whole oracle run on the
video, and the footprint reconstruction by stage isolation on the session's
own summaries: same components, same number of footprints, mask IoU >= 0.99.
"""
import numpy as np
import pytest

import oracle
from paper_2403_16438_amd import abi, segment_video

from parity import check_against_full_oracle, check_finalize_stage_isolation, params_from_config, session_outputs
from scenes import ring_video

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("path", [abi.SEG_NMF_SPLIT, abi.SEG_NMF_SINGLE], ids=["split", "single"])
@pytest.mark.parametrize("n", [3, 4, 5, 6, 7, 8])
def test_rank_n_component(n, path):
    frames = 1000 if n <= 6 else 1600
    video = ring_video(n_cells=n, radius=7.0 if n <= 6 else 8.0, frames=frames)
    sess = segment_video(video, nmf_path=path, nmf_max_rank=max(6, n))
    prm = params_from_config(sess.cfg)
    ref = oracle.segment(video, prm)
    assert ref.n_comp == 1
    assert len(ref.footprints) == n                       # the oracle's rank
    out = session_outputs(sess)
    assert check_against_full_oracle(out, ref, prm) == 0
    check_finalize_stage_isolation(out, prm)
    prof = sess.profile()
    assert prof["nmf_path"] == path
    assert prof["max_rank"] == n
    assert out["fp"]["masks"].shape[0] == n
    sess.close()
