"""MI355X (gfx950) Riesz-map solver for the high-order de Rham complex.

* ``paper_2506_17406_amd.rz``        -- ctypes binding of the HIP library
  (loads librz.so; fails loudly when it is not built);
* ``paper_2506_17406_amd.workloads`` -- seeded synthetic meshes and load vectors;
* ``paper_2506_17406_amd.build``     -- hipcc build of librz.so for gfx950.

The package import itself loads nothing, so the input generators stay usable
on machines without the library.
"""
