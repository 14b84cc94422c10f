"""MI355X-native dynamic coherence-based EM ray tracer (Wang & Manocha, DCEM).

The per-frame hot path (BVH refit, FP32 ray shooting with specular reflections,
receiver-sphere capture, FP64 image-method refinement, coherent power
accumulation and frame-to-frame path reuse) runs in hand-written HIP kernels
behind the C ABI declared in ``include/dcem.h``; ``paper_2112_07115_amd.dcem``
is the thin Python binding.  ``paper_2112_07115_amd.scenes`` builds seeded
synthetic inputs.
"""
