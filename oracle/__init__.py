"""FP64 CPU oracle of the perspective-correct hybrid-transparency splat renderer
(Hahlbohm et al., "Efficient Perspective-Correct 3D Gaussian Splatting Using
Hybrid Transparency", arXiv 2410.08129).

TEST INFRASTRUCTURE ONLY. Nothing in the product package imports, calls or
links this package; only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark do. It shares no code with the HIP path.

It is a plain, slow, brute-force renderer written in float64 PyTorch CPU ops
(so that autograd yields the float64 gradient): every Gaussian is evaluated
at every pixel ray, each pixel's fragments are fully sorted, and the hybrid
transparency formula is applied. Each function cites the passage of the
paper it follows.

Modules
  splat   activations, T, T' = VPMT, opacity-aware cutoff, screen bbox (Sec. 3.2)
  sh      real spherical-harmonics colour (Sec. 3.1, "identical to 3DGS")
  rays    pixel planes, Pluecker coordinates, rho^2, depth (Sec. 3.2, 3.3)
  blend   hybrid-transparency composite (Sec. 3.3)
  render  the brute-force renderer and crop culling
  bins    the tile/key-list reference (bbox -> pixel-centre rect -> tiles)
  densify training-side quantities beside the renderer: the densification
          statistic of the splat means and the opacity decay (Sec. 4.2)
"""
from . import splat, sh, rays, blend, render, bins, densify  # noqa: F401
