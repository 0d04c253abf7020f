"""MI355X-native (gfx950) photometry hot path: mesh background, matched-filter
detection with connected components and moments, exact-overlap aperture
photometry.  The compute lives in libgpphot.so (HIP); see include/gp.h."""
from ._lib import (GP_OK, GP_ERR_INVALID_ARG, GP_ERR_UNSUPPORTED, GP_ERR_WORKSPACE, GP_ERR_CAPACITY,
                   GP_ERR_HIP, GP_U16, GP_F32, GP_PREC_F32, GP_PREC_F64, GpError, load)

__all__ = ["GP_OK", "GP_ERR_INVALID_ARG", "GP_ERR_UNSUPPORTED", "GP_ERR_WORKSPACE", "GP_ERR_CAPACITY",
           "GP_ERR_HIP", "GP_U16", "GP_F32", "GP_PREC_F32", "GP_PREC_F64", "GpError", "load"]
