"""Plain FP64 CPU oracle for the Monte Carlo assembly of the PDDSparse system G u = b.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: it exists so that ``tests/``, the smoke check and the
CPU baseline of the benchmark can compare the HIP implementation against a
slow, obviously correct restatement of the method (Bernal, Moron-Vidal and
Acebron, "A hybrid probabilistic domain decomposition algorithm suited for
very large-scale elliptic PDEs", arXiv 2301.05780).

It shares no code with the HIP path.  Every function cites the passage of the
paper it follows; where the paper is silent the docstring names the reading
taken.  All floating point work is NumPy float64.

Modules
  philox    counter-based Philox4x32-10 stream, uniforms, Box-Muller normals
  geometry  knots, slabs/patches, sides, segment stencils, CSR pattern (Sec. 3.1)
  coeffs    the BVP coefficient families of problem (6)
  assemble  Euler-Maruyama / Gobet-Menozzi paths and the rows of G, b (eqs. 9, 20-25)
  solve     linear solve of G u = b and interface errors
  mlp       2-64-64-1 tanh network v(x) for the martingale control variate (eqs. 11, 37-38)
  evaluate  point values inside the subdomains from the knot values (eq. 8 on each square, Sec. 3.3)
  calibrate Phase II: mixed GM/EM trajectories, bias, variance, correlation, h_i and N_i (eqs. 32-41)
"""
