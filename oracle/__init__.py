"""CPU oracle for differentiable pre-filtered shadow mapping (Worchel & Alexa,
"Differentiable Shadow Mapping for Efficient Inverse Graphics", CVPR 2023).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or run
anything in this package; only the tests, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP library or its
Python binding; the only thing both sides read is the seeded input module
``scenegen``.

Structure (each step cites the passage it follows):

* ``cameras``  -- light cameras (Sec. 3 projective map L; supplementary
  renderer details) and viewer cameras, float64 torch.
* ``raster``   -- the discrete part: FP32 vertex transform with a fixed
  operation order, fixed-point snapping, brute-force coverage and the
  depth|triangle-id minimum of Eq. (1); the antialiasing edge decisions.
  numpy float32 / int64, elementwise only.
* ``mesh``     -- edge adjacency used for silhouette tests.
* ``pipeline`` -- the continuous part in float64 torch with autograd:
  moments (Alg. 1, Eq. moment1/moment2), smoothing, filtering, bilinear
  fetch, Chebyshev visibility (Sec. 3, Alg. 2), Lambert shading summed over
  lights, edge antialiasing of the image, MSE loss.  Gradients are autograd's,
  with the discrete decisions of ``raster`` held fixed.
* ``raycast``  -- brute-force float64 ray/triangle tests used only as pins.
"""
