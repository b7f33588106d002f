"""MI355X (gfx950) matrix exponential by scaling and squaring with the product-reduced Taylor
polynomials of Bader, Blanes and Casas.  The compute path is the HIP library ``libexpm.so``
(C ABI in include/expm.h); this package holds its Python binding."""
from .expm import (batched, batched_noalloc, batched_uniform, magnus4_step, select, select_rule, taylor, theta,  # noqa: F401
                   workspace_bytes)
