"""MI355X-native canonical-Huffman decoding of SZ-style uint16 quantization codes.

The compute path is the C-ABI library ``libhd.so`` (include/hd.h: host codebook
builder and reference encoder, HIP kernels for gfx950).  ``hd`` is its Python
binding; import it explicitly (``from paper_2201_09118_amd import hd``) -- it
raises when the library has not been built.
"""
