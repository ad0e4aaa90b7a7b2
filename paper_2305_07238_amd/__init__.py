"""Progressive material caching on MI355X: a HIP library behind a C ABI.

``binding`` loads the native library (``libpmc.so``) and exposes its entry
points; ``scenes`` produces seeded synthetic inputs.
"""
