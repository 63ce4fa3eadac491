"""MI355X-native range-separated (RS) canonical/Tucker assembly of N-particle
potentials, after Benner, Khoromskaia and Khoromskij (arXiv 1606.09218).

The compute path is the HIP library librs.so (C ABI in include/rs.h); this
package is its Python binding.  Importing it fails if the library is not built.
"""
from ._lib import (EXPORTED, KERNELS, PRECS, RS_E_INVALID, RS_E_RANK_CAP, RS_E_UNSUPPORTED,
                   RS_OK, Context, Factors, RSError, Tensor, assemble, energy, energy_forces,
                   energy_forces_noalloc, dot, eval_gradient_points, eval_points, gradient_grid, rbf_matvec, tensor_grid,
                   footprint_bytes, forces, make_aopts, tensor_export, tensor_load, tensor_save,
                   weighted_gram)

__all__ = ["Context", "Factors", "Tensor", "RSError", "assemble", "energy", "energy_forces",
           "energy_forces_noalloc", "dot", "eval_gradient_points", "eval_points", "gradient_grid", "rbf_matvec", "tensor_grid",
           "forces", "footprint_bytes", "make_aopts", "tensor_export", "tensor_load",
           "tensor_save", "weighted_gram", "EXPORTED", "KERNELS", "PRECS", "RS_OK",
           "RS_E_INVALID", "RS_E_RANK_CAP", "RS_E_UNSUPPORTED"]
