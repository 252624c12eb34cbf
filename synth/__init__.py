"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark: mechanism files and reactor-field generators. Nothing here
evaluates the chemistry being integrated."""
