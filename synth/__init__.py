"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

The paper's echo volumes are private (Dataset section), so every input here is
synthetic, with the shapes of Table 1 and the structure described by the
workload configurations: thick ellipsoidal LV shells, speckled chamber /
myocardium intensity volumes cropped to an apical cone, and a contracting LV
sequence.

This module holds none of the registration method's arithmetic.  Shapes are
rasterised analytically at voxel centres, rotations come from
``scipy.spatial.transform.Rotation`` and intensity resampling from
``scipy.ndimage.map_coordinates``; the HIP path and the oracle each implement
their own transform, warp and score.
"""

from .volumes import (  # noqa: F401
    gt_matrix,
    lv_sequence,
    mask_pair,
    shell_pair,
    speckle_pair,
    batch_pairs,
    make_batch_pair,
    proposal_pair,
    lv_train_pair,
)
