"""FP64 CPU oracle for the G4 slice accumulation.

TEST INFRASTRUCTURE ONLY: only the tests, the package smoke check and the
benchmark's CPU-baseline leg may import, call, link or run anything here.  The
product path (the HIP library and its Python binding) never touches it, and it
shares no code with that path.

- ``g4_oracle.c``   the plain definition in C, full-slice and entry-list modes;
- ``ref``           ctypes wrapper of it;
- ``sampled``       the same definition per entry in numpy, regenerating the
                    needed G elements from the seeded input generator, for
                    slices too large to hold G for every measurement.
"""
