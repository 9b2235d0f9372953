"""MI355X (gfx950) training path of the rank-based pseudoinverse ELM.

The product is libelm.so (HIP kernels behind the C ABI in include/elm.h);
`paper_2011_02436_amd.elm` is its Python binding and imports only when the
library has been built (`paper_2011_02436_amd.build.build()`).
"""
