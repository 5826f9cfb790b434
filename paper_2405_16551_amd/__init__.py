"""MI355X (gfx950) DE/rand/1/bin: HIP kernels behind the C ABI of include/de.h.

``paper_2405_16551_amd.de`` binds libde.so (import fails loudly if it is not
built); ``paper_2405_16551_amd.instances`` draws seeded shift/rotation data.
"""
__all__ = ["de", "instances", "build"]
