"""MI355X-native grad-h SPH hot path (GANDALF, arXiv:1709.04488, section 2.1).

``sph`` is the ctypes binding of libsph.so (HIP kernels for gfx950);
``workloads`` draws the seeded synthetic particle sets.  Importing the
package does not load the library; the binding loads it on first use and
raises if it has not been built.
"""
__all__ = ["sph", "workloads"]
