"""MI355X (gfx950) all-sky string ISW map maker: libcsmap and its binding.

The computation (paper Sec. II.A, Eq. (1)-(2), on the HEALPix sky of
Sec. II.D) runs in hand-written HIP kernels behind the C ABI of
``include/csmap.h``; this package holds those sources, their build script,
the ctypes binding and a torch.autograd wrapper.
"""
from .binding import (CSMAP_F32, CSMAP_F64, CSMAP_FORM_FP32C, CSMAP_FORM_FP64,  # noqa: F401
                      CSMAP_OPT_ACCUM, CSMAP_OPT_ADJ_SPLIT, CSMAP_OPT_BLOCK_RINGS,
                      CSMAP_OPT_CHUNK, CSMAP_OPT_FAR_W, CSMAP_OPT_GRAPH, CSMAP_OPT_NEAR_W,
                      CSMAP_OPT_PIX_PER_LANE, CSMAP_OPT_SCHEDULE, CSMAP_OPT_TILING,
                      CSMAP_OPT_WAVES, CSMAP_VIS_ALL, CSMAP_VIS_BOX, CSMAP_VIS_CAP, CsmapError,
                      Sky, pix2vec_ring)

# The differentiable map (torch.autograd.Function over render/backward) lives
# in paper_1204_5041_amd.autograd: render(sky, boxes) and StringMap.
