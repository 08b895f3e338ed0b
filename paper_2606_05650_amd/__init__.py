"""MI355X-native hot path of the GS-NFS Gaussian-frame codec.

The codec itself is libgsc.so (HIP kernels for gfx950 behind the C ABI in include/gsc.h);
`gsc` is its Python binding and `synth` the seeded synthetic-frame generator. Importing the
package loads nothing: the library is loaded on first use.
"""
