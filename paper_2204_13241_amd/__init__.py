"""MI355X (gfx950) direct X-ray speckle intensity, XPCS g2 and XSVS contrast.

Implements the direct method of arXiv:2204.13241 (Sec. 3.1, Algorithm 1) and
the reductions of Sec. 2.3 as hand-written HIP kernels behind the C ABI of
include/xs.h; this package is the thin Python binding.

    from paper_2204_13241_amd import intensity, intensity_grad, g2_rings, xsvs_contrast
"""
__all__ = [
    "intensity", "intensity_systems", "intensity_grad", "g2_rings", "xsvs_contrast",
    "IntensityFn", "make_batch", "get_tile_shape", "set_tile_shape", "shutdown", "inputs",
    "speckle_loss", "position_step", "timing_enable", "timing_read", "roofline_probe", "Plan",
]


def __getattr__(name):
    # The binding (and torch) load on first use, so the input generators can be
    # imported on machines without the built library.
    import importlib
    if name in ("inputs", "api", "build"):
        return importlib.import_module(__name__ + "." + name)
    if name in __all__:
        return getattr(importlib.import_module(__name__ + ".api"), name)
    raise AttributeError(name)
