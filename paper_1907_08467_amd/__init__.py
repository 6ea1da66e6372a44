"""vcs355: batched Atari 2600 emulation on one MI355X (gfx950).

The HIP library (libvcs355.so, C ABI in include/vcs355.h) is loaded by
`paper_1907_08467_amd.binding`; `paper_1907_08467_amd.env.VcsEnv` is the
torch-facing wrapper.  Importing this package itself loads nothing, so the
seeded input generators in `paper_1907_08467_amd.inputs` work without a GPU.
"""
