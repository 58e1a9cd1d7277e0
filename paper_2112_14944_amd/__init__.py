"""MI355X (gfx950) PPR -> DPPR -> PDist -> stress-layout library.

The computation runs in libpprviz.so (hand-written HIP, see csrc/); this
package only marshals torch tensors into its C ABI (include/pprviz.h).
Import `paper_2112_14944_amd.ops` for the calls and
`paper_2112_14944_amd.autograd` for the differentiable loss.
"""
__all__ = ["ops", "autograd", "build"]
