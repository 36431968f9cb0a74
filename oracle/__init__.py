"""Plain, slow CPU oracle for the occupancy-plane ray marcher (TEST INFRASTRUCTURE).

This package is test infrastructure.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it.  The product path
(``paper_2404_09531_amd``) never imports, calls or links anything here, and
this package imports nothing from the product path; the two share only the
seeded input generators in ``scenegen``.

What it computes (Oblique-MERF, arXiv 2404.09531):

* sample placement inside the occupancy plane's intervals (Sec. 4.1,
  Eq. 6 at epsilon = 0, Eq. 7; Sec. 4.4 "sample only inside
  [z_min, z_max]") -- ``placement.py``;
* MERF features: trilinear grid + three bilinear planes (Sec. 3, Eq. 2) and
  their activations (Eq. 3) -- ``field.py``;
* volume-rendering quadrature (Eq. 1), deferred MLP (Eq. 4), the soft
  occupancy value (Eq. 6, 8), the L2 loss with its float64 autograd
  gradient, the interval-span loss (Eq. 5), the view-direction encoding of
  the deferred MLP and the view-smoothness loss (Eq. 9-10) -- ``render.py``;
* 8-bit storage of the baked features (Sec. 4.4) -- ``quant.py``.

Precision: float64 throughout, except the placement predicate, which is
defined in binary32 (see ``placement.py``), and the 8-bit code decision
(see ``quant.py``), so that both sides take each discrete decision in the
same precision.

Every function cites the passage it follows.  Readings of silent or
ambiguous passages are listed in the module docstrings where they apply.
"""
from .placement import (K_CAP, box_k_interval, cell_index, lattice_points,
                        place_samples, accept_mask)
from .field import interp_features, activations, corner_weights_1d
from .render import (RenderParams, oracle_render, oracle_loss_and_grads,
                     mlp_forward, composite, occupancy_value, occ_interval_loss,
                     encode_dir, smooth_loss)
from .quant import (feature_range, quant_params, quantize_u8, dequantize, quantize_scene,
                    dequantize_scene)

__all__ = [
    "K_CAP", "box_k_interval", "cell_index", "lattice_points", "place_samples",
    "accept_mask", "interp_features", "activations", "corner_weights_1d",
    "RenderParams", "oracle_render", "oracle_loss_and_grads", "mlp_forward",
    "composite", "occupancy_value", "occ_interval_loss", "encode_dir", "smooth_loss",
    "feature_range", "quant_params", "quantize_u8", "dequantize", "quantize_scene", "dequantize_scene",
]
