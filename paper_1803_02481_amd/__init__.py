"""hipbmg: structured variational multigrid for 2D heterogeneous diffusion on
AMD MI355X (gfx950), after Reisner, Olson and Moulton (arXiv 1803.02481).

The compute path is the C-ABI library ``libhipbmg.so`` (hand-written HIP);
``paper_1803_02481_amd.hipbmg`` is its thin Python binding.  Importing this
package loads nothing: the binding loads the library on first use and raises if
it is missing.
"""
__all__ = ["hipbmg", "inputs"]
