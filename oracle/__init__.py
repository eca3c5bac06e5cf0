"""Plain FP64 CPU oracle of the TRINITY time-dependent radiative-transfer step.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path (the
HIP library and its Python binding) never imports, links or calls it, and it
shares no code with that path: no kernels, headers, tables or helpers.

Every function cites the part of the paper (Yajima et al., "TRINITY: a
three-dimensional time-dependent radiative transfer code for in-vivo
near-infrared imaging") that it follows.  The code is written for a reader
checking it against the paper by eye: no blocking, fusion or reordering
beyond what the equations state.  Readings of passages the paper leaves open
are marked "Reading:" where they are used.

Modules
  angles   HEALPix directions, Henyey-Greenstein phase matrix, Eq. (9) weights
  medium   time step, path length per step, collision coefficients
  lattice  long-characteristic ray lattice: dominant axis, plane shifts, move fraction
  optics   Snell's law, Fresnel reflectance, interface interception lists
  setup    source and detector sets, pulse weights, rebinning
  solve    the forward step loop (injection, collision, transport, tallies)
  adjoint  exact transpose of the step loop and the per-voxel gradient
  physics  closed forms used as pins (random walk, diffusion decay)
"""
