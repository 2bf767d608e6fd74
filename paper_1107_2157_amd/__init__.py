"""MI355X-native two-step Lax-Wendroff shallow-water library (libsw).

``paper_1107_2157_amd.sw`` is the ctypes binding of the C ABI in
``include/sw.h``; ``paper_1107_2157_amd.ics`` holds the seeded initial
states; ``paper_1107_2157_amd.build`` compiles the HIP library in-tree.
Importing the package loads nothing; the library is loaded on first use.
"""
__all__ = ["sw", "ics", "build"]
