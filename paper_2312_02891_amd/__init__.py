"""MI355X-native inexact low-rank Sylvester ADI (see include/lradi.h).

Importing the package loads nothing native; `paper_2312_02891_amd.lradi`
loads the HIP library and fails loudly when it is missing.
"""
