"""MI355X-native hot path of holistic bundle adjustment (one LM iteration).

The compute path is libba.so (HIP for gfx950, C ABI in include/ba.h);
``paper_2609_04026_amd.binding`` is its ctypes binding.  Importing this
package does not load the library; importing ``binding`` does, and fails
loudly when it is not built.
"""
