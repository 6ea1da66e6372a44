"""Seeded input generators shared by the CPU oracle and the GPU path.

Nothing here emulates anything: the assembler and cartridge generator produce
ROM bytes, the palette module produces the gray table, and ``workloads``
produces env-to-ROM assignments and action streams.
"""
