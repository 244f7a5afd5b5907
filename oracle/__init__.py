"""FP64 CPU reference for the position-dependent (smearing-distorted) PSF.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The GPU
library (``paper_2009_07010_amd``) never imports, links or calls it, and this
package imports nothing from the library; the two share only the seeded
input generator ``psf_synth``, which holds none of the method's arithmetic.

Every function computes the plain definition in float64 / complex128 and
cites the passage of Atemkeng et al. (2020), "Fast algorithms to approximate
the position-dependent point spread function responses in radio
interferometric wide-field imaging", that it follows.  See ``psf64`` for the
readings taken where the paper is silent.
"""
from .psf64 import (  # noqa: F401
    C_LIGHT, BinTable, bin_table, bin_centres_lambda, decorr, decorr_sinc, decorr_with_grad,
    decorr_brute, wshift, pixel_offsets, patch_factored, patch_brute, patch_pixels,
    patch_fullw, patch_fullw_pixels, patch_normalised, peak_normalised_error, loss_value,
    loss_grad_analytic, loss_grad_fd, hogbom_clean, hogbom_clean_method2, OMEGA_EARTH, method2_grid, method2_dhat,
    method2_effective_psf, method2_patch,
)
