"""MI355X-native hot path of the Ray Theory of Waves (Ren et al., arXiv 2403.13856).

Rays traced through a smooth ellipsoid carry a 2x2 wavefront-curvature matrix
updated by the paper's wavefront equation (Eq. 3) at each reflection and
refraction; their far-field amplitude and phase are summed coherently on a
(theta, phi) grid.  The work runs in hand-written HIP kernels behind the C ABI
declared in ``include/rtw.h``; ``paper_2403_13856_amd.rtw`` is its thin Python
binding (argument marshalling only).
"""
__all__ = ["inputs"]
