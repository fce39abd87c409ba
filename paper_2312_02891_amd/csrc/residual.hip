// filled in later
