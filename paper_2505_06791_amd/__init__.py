"""MI355X-native batched motion projection and validation for constrained
bidirectional RRT-Connect (cpRRTC, arXiv 2505.06791).

Importing the package loads nothing; `paper_2505_06791_amd.cprrtc` binds the
HIP library (libcprrtc.so) and `paper_2505_06791_amd.inputs` draws seeded
synthetic robots, scenes and configurations.
"""
