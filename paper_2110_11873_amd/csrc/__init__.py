"""HIP sources of librt.so and their build script."""
