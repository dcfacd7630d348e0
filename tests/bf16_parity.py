"""Element-wise comparison of a BF16-network result computed on the GPU with the oracle in bf16 mode.

Both sides round weights, activations and back-propagated signals to BF16 at the same points; the GPU
sums in FP32, the oracle in FP64.  An element whose inputs rounded alike differs only by the FP32
summation, far below one BF16 ulp (2^-8 relative): it lies within `tight` x scale.  Where an FP32 sum
sits within its rounding error of a BF16 rounding boundary, the two sides round that activation to
neighbouring BF16 values (a flip), and the elements downstream of it differ by up to a few ulps: they
must lie within `loose` x scale, and they may make up at most `max_flip_frac` of the elements, or the
footprint of one flip where that is more (an activation feeds at most 9 x 9 outputs through the three
3 x 3 layers after it).  Scale is the largest magnitude of the reference.
"""
import numpy as np

ULP = 2.0 ** -8          # one BF16 ulp, relative
TIGHT = ULP / 16         # FP32-versus-FP64 summation, inputs rounded alike
LOOSE = 4 * ULP          # downstream of a flipped rounding


FOOTPRINT = 81


def elementwise(got, ref, what, tight=TIGHT, loose=LOOSE, max_flip_frac=0.05, footprint=FOOTPRINT):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    scale = max(float(np.max(np.abs(ref))), 1e-300)
    err = np.abs(got - ref) / scale
    worst = float(err.max()) if err.size else 0.0
    flips = int(np.count_nonzero(err > tight))
    print(f"{what}: max |diff| {worst:.3e} x scale, {flips} of {err.size} beyond {tight:.1e}")
    assert np.all(np.isfinite(got)), f"{what}: non-finite values"
    assert worst <= loose, f"{what}: max |diff| = {worst:.3e} x scale > {loose:.1e}"
    allowed = max(max_flip_frac * err.size, footprint)
    assert flips <= allowed, f"{what}: {flips} of {err.size} elements beyond {tight:.1e} x scale (allowed {allowed:.0f})"
    return worst, flips
