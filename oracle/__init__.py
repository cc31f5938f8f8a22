"""FP64 CPU oracle (test infrastructure only; see hh_ref)."""
from .hh_ref import (chirp, fresnel_ref, space_time_matrix, covariance_ref, phase_fix,
                     eigh_ref, project_render_ref, pipeline_ref, dft_basis,
                     fourier_render_ref, svd_filter_ref, covariance_frames_ref, project_first_ref,
                     pipeline_first_ref, PHASE_TIE_REL)
