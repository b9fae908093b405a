"""Seeded synthetic inputs shared by the CPU oracle tests and the HIP path."""
